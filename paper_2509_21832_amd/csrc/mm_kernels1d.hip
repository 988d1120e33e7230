// mm_kernels1d.hip -- 1D1V BGK micro-macro step on gfx950 (FP64).
//
// Paper: Rossmanith & Sar, arXiv:2509.21832, Sec. 3.3 (micro update
// eqn5-19 .. eqn5-25 with periodic / extrapolation ghosts) and Sec. 3.4
// (heat flux eqn5-26, KFVS macro update eqn5-27, flux1d_1/2).
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

__device__ __forceinline__ int nbr1(const Params &P, int i, int up)
{
    if (up) return i < P.nx - 1 ? i + 1 : (P.bc[1].kind == BC_PERIODIC ? 0 : i);
    return i > 0 ? i - 1 : (P.bc[0].kind == BC_PERIODIC ? P.nx - 1 : i);
}

// one workgroup per cell: G^n -> G^{n+1} (eqn5-25) and H^{n+1} (eqn5-26)
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_micro1d(const double *__restrict__ Q, const double *__restrict__ G,
                                                    double *__restrict__ Gn, double *__restrict__ H, Params P)
{
    __shared__ double lds[NW * 12];
    const int i = blockIdx.x;
    const Prim1 s = prim1(Q + 3 * (size_t)i);
    const Prim1 sm = prim1(Q + 3 * (size_t)nbr1(P, i, 0));
    const Prim1 sp = prim1(Q + 3 * (size_t)nbr1(P, i, 1));
    const double tau = tau_of(P, s.rho, s.rho * s.T, s.T);
    const double Tiph = 0.5 * (sp.T + s.T), Timh = 0.5 * (sm.T + s.T);
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
    // sums: phi.Z (3), phi.Gh (3), Gram (6: 00 01 02 11 12 22)
    double sm_[12];
#pragma unroll
    for (int n = 0; n < 12; ++n) sm_[n] = 0.0;
    for (int k = threadIdx.x; k < P.nv1; k += 64 * NW) {
        double Z, M, Gh, f1, f2, gc;
        point(k, Z, M, Gh, f1, f2, gc);
        sm_[0] += Z; sm_[1] += f1 * Z; sm_[2] += f2 * Z;
        sm_[3] += Gh; sm_[4] += f1 * Gh; sm_[5] += f2 * Gh;
        sm_[6] += M; sm_[7] += f1 * M; sm_[8] += f2 * M;
        sm_[9] += f1 * f1 * M; sm_[10] += f1 * f2 * M; sm_[11] += f2 * f2 * M;
    }
    block_sum<12, NW>(sm_, lds);
    double AZ[3], AG[3] = {0.0, 0.0, 0.0};
    if (P.proj_mode == PROJ_PAPER) {
        for (int a = 0; a < 3; ++a) AZ[a] = P.dv1 / s.rho * sm_[a];
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
        }
    }
    const double ra = P.eps / (P.eps + P.dt * tau), rb = P.dt * tau / (P.eps + P.dt * tau);
    double hs[1] = {0.0};
    for (int k = threadIdx.x; k < P.nv1; k += 64 * NW) {
        double Z, M, Gh, f1, f2, gc;
        point(k, Z, M, Gh, f1, f2, gc);
        const double PZ = (AZ[0] + AZ[1] * f1 + AZ[2] * f2) * M;
        const double PG = (AG[0] + AG[1] * f1 + AG[2] * f2) * M;
        const double gn = ra * (gc - P.dt * (Z - PZ)) + rb * (Gh - PG);
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

// Q^n -> Q^{n+1} (eqn5-27)
__global__ void k_macro1d(const double *__restrict__ Q, const double *__restrict__ H, double *__restrict__ Qn,
                          int *__restrict__ flag, int step, Params P)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.nx) return;
    double FL[3], FR[3], HL, HR;
    face1(P, Q, H, i, FL, HL);
    face1(P, Q, H, i + 1, FR, HR);
    double q[3];
    for (int r = 0; r < 3; ++r) q[r] = Q[3 * (size_t)i + r] - P.dt / P.dx * (FR[r] - FL[r]);
    q[2] -= P.dt / P.dx * (HR - HL);
    const Prim1 s = prim1(q);
    if (!(s.rho > 0.0) || !(s.T > 0.0) || !isfinite(s.u)) atomicMin(flag, step + 1);
    for (int r = 0; r < 3; ++r) Qn[3 * (size_t)i + r] = q[r];
}

void launch_step1d(const double *Q, double *Qn, const double *G, double *Gn, double *H, int *flag, int step,
                   const Params &P, hipStream_t st)
{
    hipLaunchKernelGGL(k_micro1d<2>, dim3(P.nx), dim3(128), 0, st, Q, G, Gn, H, P);
    hipLaunchKernelGGL(k_macro1d, dim3((P.nx + 127) / 128), dim3(128), 0, st, Q, H, Qn, flag, step, P);
}

} // namespace mm
