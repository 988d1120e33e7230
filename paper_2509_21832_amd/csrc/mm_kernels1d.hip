// mm_kernels1d.hip -- 1D1V BGK micro-macro step on gfx950 (FP64).
//
// Paper: Rossmanith & Sar, arXiv:2509.21832, Sec. 3.3 (micro update
// eqn5-19 .. eqn5-25 with periodic / extrapolation ghosts) and Sec. 3.4
// (heat flux eqn5-26, KFVS macro update eqn5-27, flux1d_1/2); diffusely
// reflecting walls of Sec. 4.3 (wall_bc_1/2).
#include "mm_device.h"
#include "mm_launch.h"

namespace mm {

struct Prim1 {
    double rho, u, T;
};

__device__ __forceinline__ Prim1 prim1(const double *q)
{
    Prim1 s;
    s.rho = q[0];
    s.u = q[1] / q[0];
    s.T = 2.0 * q[2] / q[0] - s.u * s.u;     // E = rho T/2 + rho u^2/2
    return s;
}

// Diffuse wall on side 0 (x_lo, emitting into v > 0) or 1 (x_hi, into v < 0) next
// to a cell in state s (Sec. 4.3).  Half-range moments of the cell's Maxwellian,
// with a = sqrt(T / 2 pi) exp(-u^2 / 2T) and b+- = (1 +- erf(u / sqrt(2T))) / 2:
//   toward the x_lo wall (v < 0): mass rho b-, flux rho (u b- - a), second moment
//   rho ((T + u^2) b- - u a); toward the x_hi wall (v > 0): rho b+, rho (u b+ + a),
//   rho ((T + u^2) b+ + u a).
struct Wall1 {
    double rho;    // wall density: its half flux rho sqrt(T_w / 2 pi) cancels the cell's
    double T;      // interface temperature: second over zeroth moment of the
                   // wall-half / cell-half distribution
};
__device__ __forceinline__ Wall1 wall1(const Prim1 &s, double T_w, int side)
{
    const double a = sqrt(s.T / (2.0 * MM_PI)) * exp(-s.u * s.u / (2.0 * s.T));
    const double er = erf(s.u / sqrt(2.0 * s.T));
    const double b = side == 0 ? 0.5 * (1.0 - er) : 0.5 * (1.0 + er);
    const double ua = side == 0 ? -s.u * a : s.u * a;          // the signed u a term
    const double flux = side == 0 ? a - s.u * b : a + s.u * b;  // |mass flux toward the wall| / rho
    Wall1 w;
    w.rho = s.rho * flux * sqrt(2.0 * MM_PI / T_w);
    w.T = (s.rho * ((s.T + s.u * s.u) * b + ua) + 0.5 * w.rho * T_w) / (s.rho * b + 0.5 * w.rho);
    return w;
}

__device__ __forceinline__ int nbr1(const Params &P, int i, int up)
{
    if (up) return i < P.nx - 1 ? i + 1 : (P.bc[1].kind == BC_PERIODIC ? 0 : i);
    return i > 0 ? i - 1 : (P.bc[0].kind == BC_PERIODIC ? P.nx - 1 : i);
}

// The manufactured solution of the 1D convergence study (Sec. 3.4):
//   f = A(v) B(t, x),  A = exp(-(v - 1)^2) + 2 exp(-(v + 1)^2),  B = 2 + sin 2pi(x - t),
// with rho = 3 sqrt(pi) B, u = -1/3, T = 25/18, so its Maxwellian is
// 1.8 exp(-0.04 (3v + 1)^2) B and its micro part g = (f - M) / eps.  Its residual
//   S = f_t + v f_x - (tau / eps)(M - f) = 2 pi cos 2pi(x - t) (v - 1) A + tau g,
// with tau the cell's tau_i^n, enters G-hat as (1 / tau)(I - Pi)[S], and the macro
// update as dt int (1, v, v^2 / 2) S dv = dt pi^(3/2) cos 2pi(x - t) (-8, 11, -7).
__device__ __forceinline__ double mms1_S(double eps, double tau, double t, double x, double v)
{
    const double ph = 2.0 * MM_PI * (x - t);
    const double A = exp(-(v - 1.0) * (v - 1.0)) + 2.0 * exp(-(v + 1.0) * (v + 1.0));
    const double g = (A - 1.8 * exp(-0.04 * (3.0 * v + 1.0) * (3.0 * v + 1.0))) * (2.0 + sin(ph)) / eps;
    return 2.0 * MM_PI * cos(ph) * (v - 1.0) * A + tau * g;
}

// one workgroup per cell: G^n -> G^{n+1} (eqn5-25) and H^{n+1} (eqn5-26); with mms
// set, plus the manufactured-solution source at time t
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_micro1d(const double *__restrict__ Q, const double *__restrict__ G,
                                                    double *__restrict__ Gn, double *__restrict__ H, Params P,
                                                    int mms, double t)
{
    __shared__ double lds[NW * 15];
    const int i = blockIdx.x;
    const Prim1 s = prim1(Q + 3 * (size_t)i);
    const Prim1 sm = prim1(Q + 3 * (size_t)nbr1(P, i, 0));
    const Prim1 sp = prim1(Q + 3 * (size_t)nbr1(P, i, 1));
    const double tau = tau_of(P, s.rho, s.rho * s.T, s.T);
    double Tiph = 0.5 * (sp.T + s.T), Timh = 0.5 * (sm.T + s.T);
    if (i == 0 && P.bc[0].kind == BC_WALL) Timh = wall1(s, P.bc[0].T_wall, 0).T;
    if (i == P.nx - 1 && P.bc[1].kind == BC_WALL) Tiph = wall1(s, P.bc[1].T_wall, 1).T;
    const double dT = (Tiph - Timh) / (P.dx * s.T);
    const double mpre = s.rho / sqrt(2.0 * MM_PI * s.T), rsT = 1.0 / sqrt(s.T), r2 = sqrt(2.0);
    const size_t nv = P.nv1;
    const double *Gc = G + (size_t)i * nv;
    const double *Gm, *Gp;
    if (i > 0) Gm = Gc - nv;
    else if (P.bc[0].kind == BC_PERIODIC) Gm = Gc + (size_t)(P.nx - 1) * nv;
    else Gm = is_open(P.bc[0].kind) ? nullptr : Gc;
    if (i < P.nx - 1) Gp = Gc + nv;
    else if (P.bc[1].kind == BC_PERIODIC) Gp = Gc - (size_t)(P.nx - 1) * nv;
    else Gp = is_open(P.bc[1].kind) ? nullptr : Gc;

    auto point = [&](int k, double &Z, double &M, double &Gh, double &f1, double &f2, double &gc) {
        const double v = P.v1_lo + (k + 0.5) * P.dv1, w = v - s.u;
        M = mpre * exp(-w * w / (2.0 * s.T));
        Gh = -(1.0 / tau) * (w * w * w / (2.0 * s.T) - 1.5 * w) * dT * M;
        gc = Gc[k];
        const double gm = Gm ? Gm[k] : 0.0, gp = Gp ? Gp[k] : 0.0;
        Z = fmin(0.0, v) * ((gp - gc) / P.dx) + fmax(0.0, v) * ((gc - gm) / P.dx);
        f1 = w * rsT;
        f2 = r2 * (w * w / (2.0 * s.T) - 0.5);
    };
    const double xc = P.x_lo + (i + 0.5) * P.dx;
    // sums: phi.Z (3), phi.Gh (3), Gram (6: 00 01 02 11 12 22), phi.S (3)
    double sm_[15];
#pragma unroll
    for (int n = 0; n < 15; ++n) sm_[n] = 0.0;
    for (int k = threadIdx.x; k < P.nv1; k += 64 * NW) {
        double Z, M, Gh, f1, f2, gc;
        point(k, Z, M, Gh, f1, f2, gc);
        sm_[0] += Z; sm_[1] += f1 * Z; sm_[2] += f2 * Z;
        sm_[3] += Gh; sm_[4] += f1 * Gh; sm_[5] += f2 * Gh;
        sm_[6] += M; sm_[7] += f1 * M; sm_[8] += f2 * M;
        sm_[9] += f1 * f1 * M; sm_[10] += f1 * f2 * M; sm_[11] += f2 * f2 * M;
        if (mms) {
            const double S = mms1_S(P.eps, tau, t, xc, P.v1_lo + (k + 0.5) * P.dv1);
            sm_[12] += S; sm_[13] += f1 * S; sm_[14] += f2 * S;
        }
    }
    block_sum<15, NW>(sm_, lds);
    double AZ[3], AG[3] = {0.0, 0.0, 0.0}, AS[3];
    if (P.proj_mode == PROJ_PAPER) {
        for (int a = 0; a < 3; ++a) AZ[a] = P.dv1 / s.rho * sm_[a];
        for (int a = 0; a < 3; ++a) AS[a] = P.dv1 / s.rho * sm_[12 + a];
    } else {
        // solve the 3x3 Gram system (Cramer's rule on the symmetric matrix)
        const double g00 = sm_[6], g01 = sm_[7], g02 = sm_[8], g11 = sm_[9], g12 = sm_[10], g22 = sm_[11];
        const double c00 = g11 * g22 - g12 * g12, c01 = g02 * g12 - g01 * g22, c02 = g01 * g12 - g02 * g11;
        const double c11 = g00 * g22 - g02 * g02, c12 = g01 * g02 - g00 * g12, c22 = g00 * g11 - g01 * g01;
        const double det = g00 * c00 + g01 * c01 + g02 * c02;
        const double I[3][3] = {{c00, c01, c02}, {c01, c11, c12}, {c02, c12, c22}};
        for (int a = 0; a < 3; ++a) {
            AZ[a] = (I[a][0] * sm_[0] + I[a][1] * sm_[1] + I[a][2] * sm_[2]) / det;
            AG[a] = (I[a][0] * sm_[3] + I[a][1] * sm_[4] + I[a][2] * sm_[5]) / det;
            AS[a] = (I[a][0] * sm_[12] + I[a][1] * sm_[13] + I[a][2] * sm_[14]) / det;
        }
    }
    const double ra = P.eps / (P.eps + P.dt * tau), rb = P.dt * tau / (P.eps + P.dt * tau);
    double hs[1] = {0.0};
    for (int k = threadIdx.x; k < P.nv1; k += 64 * NW) {
        double Z, M, Gh, f1, f2, gc;
        point(k, Z, M, Gh, f1, f2, gc);
        const double PZ = (AZ[0] + AZ[1] * f1 + AZ[2] * f2) * M;
        const double PG = (AG[0] + AG[1] * f1 + AG[2] * f2) * M;
        double gh = Gh - PG;
        if (mms) {
            const double S = mms1_S(P.eps, tau, t, xc, P.v1_lo + (k + 0.5) * P.dv1);
            gh += (S - (AS[0] + AS[1] * f1 + AS[2] * f2) * M) / tau;
        }
        const double gn = ra * (gc - P.dt * (Z - PZ)) + rb * gh;
        Gn[(size_t)i * nv + k] = gn;
        const double v = P.v1_lo + (k + 0.5) * P.dv1;
        hs[0] += v * v * v * gn;
    }
    block_sum<1, NW>(hs, lds);
    if (threadIdx.x == 0) H[i] = 0.5 * P.eps * P.dv1 * hs[0];
}

// KFVS half flux of (flux1d_2): sgn +1 integrates v > 0
__device__ __forceinline__ void kfvs_half1(const double *q, double sgn, double F[3])
{
    const double rho = q[0], u = q[1] / rho, T = 2.0 * q[2] / rho - u * u;
    const double alpha = sqrt(T / (2.0 * MM_PI)) * exp(-u * u / (2.0 * T));
    const double beta = 0.5 * (1.0 + sgn * erf(u / sqrt(2.0 * T)));
    const double f[3] = {rho * u, rho * (T + u * u), 0.5 * rho * u * (3.0 * T + u * u)};
    const double m[3] = {rho, rho * u, 0.5 * rho * (2.0 * T + u * u)};
    for (int r = 0; r < 3; ++r) F[r] = sgn * alpha * m[r] + beta * f[r];
}

__device__ __forceinline__ void face1(const Params &P, const double *Q, const double *H, int f, double F[3], double &Hf)
{
    double fp[3], fm[3];
    const int nx = P.nx;
    if (f > 0 && f < nx) {
        kfvs_half1(Q + 3 * (size_t)(f - 1), 1.0, fp);
        kfvs_half1(Q + 3 * (size_t)f, -1.0, fm);
        for (int r = 0; r < 3; ++r) F[r] = fp[r] + fm[r];
        Hf = 0.5 * (H[f] + H[f - 1]);
    } else if (P.bc[0].kind == BC_PERIODIC) {
        kfvs_half1(Q + 3 * (size_t)(nx - 1), 1.0, fp);
        kfvs_half1(Q, -1.0, fm);
        for (int r = 0; r < 3; ++r) F[r] = fp[r] + fm[r];
        Hf = 0.5 * (H[0] + H[nx - 1]);
    } else if (P.bc[f == 0 ? 0 : 1].kind == BC_WALL) {
        // KFVS between the wall Maxwellian (rho_w, 0, T_w) and the edge cell; the
        // ghost's H is 0, so H_{1/2} = H_1 / 2 (Sec. 4.3)
        const int side = f == 0 ? 0 : 1, e = f == 0 ? 0 : nx - 1;
        const double *q = Q + 3 * (size_t)e;
        const double Tw = P.bc[side].T_wall;
        const Wall1 w = wall1(prim1(q), Tw, side);
        const double qw[3] = {w.rho, 0.0, 0.5 * w.rho * Tw};
        kfvs_half1(side == 0 ? qw : q, 1.0, fp);
        kfvs_half1(side == 0 ? q : qw, -1.0, fm);
        for (int r = 0; r < 3; ++r) F[r] = fp[r] + fm[r];
        Hf = 0.5 * H[e];
    } else {
        const int e = f == 0 ? 0 : nx - 1;
        const double *q = Q + 3 * (size_t)e;
        const double rho = q[0], u = q[1] / rho, T = 2.0 * q[2] / rho - u * u;
        F[0] = rho * u;
        F[1] = rho * (T + u * u);
        F[2] = 0.5 * rho * u * (3.0 * T + u * u);
        Hf = H[e];
    }
}

// Q^n -> Q^{n+1} (eqn5-27); with mms set, plus the manufactured-solution source at time t
__global__ void k_macro1d(const double *__restrict__ Q, const double *__restrict__ H, double *__restrict__ Qn,
                          int *__restrict__ flag, int step, Params P, int mms, double t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.nx) return;
    double FL[3], FR[3], HL, HR;
    face1(P, Q, H, i, FL, HL);
    face1(P, Q, H, i + 1, FR, HR);
    double q[3];
    for (int r = 0; r < 3; ++r) q[r] = Q[3 * (size_t)i + r] - P.dt / P.dx * (FR[r] - FL[r]);
    q[2] -= P.dt / P.dx * (HR - HL);
    if (mms) {
        const double src = P.dt * MM_PI * sqrt(MM_PI) * cos(2.0 * MM_PI * (P.x_lo + (i + 0.5) * P.dx - t));
        q[0] += -8.0 * src;
        q[1] += 11.0 * src;
        q[2] += -7.0 * src;
    }
    const Prim1 s = prim1(q);
    if (!(s.rho > 0.0) || !(s.T > 0.0) || !isfinite(s.u)) atomicMin(flag, step + 1);
    for (int r = 0; r < 3; ++r) Qn[3 * (size_t)i + r] = q[r];
}

void launch_step1d(const double *Q, double *Qn, const double *G, double *Gn, double *H, int *flag, int step,
                   const Params &P, hipStream_t st, int mms, double t)
{
    hipLaunchKernelGGL(k_micro1d<2>, dim3(P.nx), dim3(128), 0, st, Q, G, Gn, H, P, mms, t);
    hipLaunchKernelGGL(k_macro1d, dim3((P.nx + 127) / 128), dim3(128), 0, st, Q, H, Qn, flag, step, P, mms, t);
}

} // namespace mm
