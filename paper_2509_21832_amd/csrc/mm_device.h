// mm_device.h -- device helpers shared by the 1D and 2D kernels: block
// reductions for 64-wide wavefronts and the pointwise macro formulas.
#pragma once
#include "mm_internal.h"

namespace mm {

// Sum N doubles over a block of NW wavefronts (blockDim.x = 64 NW).  Every
// thread ends with the block totals.  Fixed combination order, so repeated
// runs are bitwise identical.  `lds` holds NW * N doubles.
template <int N, int NW>
__device__ __forceinline__ void block_sum(double (&v)[N], double *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += __shfl_xor(v[n], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int n = 0; n < N; ++n) lds[wid * N + n] = v[n];
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double s = lds[n];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += lds[w * N + n];
        v[n] = s;
    }
    __syncthreads();
}

// Cell (i, j) of the r-th wall-adjacent cell of the ring: bottom row, top
// row, then the left and right columns without their corners
__device__ __forceinline__ void ring_cell(const Params &P, int r, int &i, int &j)
{
    if (r < P.nx) { i = r; j = 0; return; }
    r -= P.nx;
    if (r < P.nx) { i = r; j = P.ny - 1; return; }
    r -= P.nx;
    if (r < P.ny - 2) { i = 0; j = r + 1; return; }
    r -= P.ny - 2;
    i = P.nx - 1;
    j = r + 1;
}

__device__ __forceinline__ double tau_of(const Params &P, double rho, double p, double T)
{
    switch (P.tau_model) {
    case TAU_RHO:  return P.tau_coef * rho;
    case TAU_P:    return P.tau_coef * p;
    case TAU_HS1D: return P.tau_coef * sqrt(T / (2.0 * MM_PI));
    default:       return P.tau_coef;
    }
}

// ---------------------------------------------------------------------------
// 2D macro pieces (Sec. 5.4)

// TR-BDF2 (gamma = 1/2) factor for the collision half step, written with dt
__device__ __forceinline__ double trbdf2_W(double eps, double tau, double nu, double dt)
{
    const double r = tau * (1.0 - nu);
    return (48.0 * eps * eps - 10.0 * r * eps * dt) /
           (48.0 * eps * eps + 14.0 * r * eps * dt + (r * dt) * (r * dt));
}

// collision half step on the pressure tensor of one cell (macro2d-split1/4)
__device__ __forceinline__ void collide(const Params &P, double q[6])
{
    const double rho = q[0], ir = 1.0 / rho, u1 = q[1] * ir, u2 = q[2] * ir;
    const double P11 = q[3] - q[1] * u1, P12 = q[4] - q[1] * u2, P22 = q[5] - q[2] * u2;
    const double p = 0.5 * (P11 + P22);
    const double W = trbdf2_W(P.eps, tau_of(P, rho, p, p * ir), P.nu, P.dt);
    const double n11 = 0.5 * ((1.0 + W) * P11 + (1.0 - W) * P22);
    const double n12 = 0.5 * (2.0 * W * P12);
    const double n22 = 0.5 * ((1.0 - W) * P11 + (1.0 + W) * P22);
    q[3] = rho * u1 * u1 + n11;
    q[4] = rho * u1 * u2 + n12;
    q[5] = rho * u2 * u2 + n22;
}

// Half-space KFVS flux of the Gaussian with the six moments of q along
// direction d (0: v1, 1: v2); sgn = +1 integrates d-velocity > 0.
// F = 1/2 (sgn a J + (1 + sgn b) K) with a, b, J, K of (flux-2D-1/2).
__device__ __forceinline__ void kfvs_half(const double q[6], int d, double sgn, double F[6])
{
    // one reciprocal each of rho and of the normal pressure instead of a division per use
    const double rho = q[0], ir = 1.0 / rho, u1 = q[1] * ir, u2 = q[2] * ir;
    const double P11 = q[3] - q[1] * u1, P12 = q[4] - q[1] * u2, P22 = q[5] - q[2] * u2;
    double a, b, J[6], K[6];
    if (d == 0) {
        const double iP = 1.0 / P11;
        a = sqrt((2.0 / MM_PI) * P11 * ir) * exp(-0.5 * rho * u1 * u1 * iP);
        b = erf(u1 * sqrt(0.5 * rho * iP));
        J[0] = rho; J[1] = rho * u1; J[2] = rho * u2;
        J[3] = rho * u1 * u1 + 2.0 * P11;
        J[4] = rho * u1 * u2 + 2.0 * P12;
        J[5] = rho * u2 * u2 + P22 + P12 * P12 * iP;
        K[0] = rho * u1;
        K[1] = rho * u1 * u1 + P11;
        K[2] = rho * u1 * u2 + P12;
        K[3] = rho * u1 * u1 * u1 + 3.0 * u1 * P11;
        K[4] = rho * u1 * u1 * u2 + u2 * P11 + 2.0 * u1 * P12;
        K[5] = rho * u1 * u2 * u2 + u1 * P22 + 2.0 * u2 * P12;
    } else {
        const double iP = 1.0 / P22;
        a = sqrt((2.0 / MM_PI) * P22 * ir) * exp(-0.5 * rho * u2 * u2 * iP);
        b = erf(u2 * sqrt(0.5 * rho * iP));
        J[0] = rho; J[1] = rho * u1; J[2] = rho * u2;
        J[3] = rho * u1 * u1 + P11 + P12 * P12 * iP;
        J[4] = rho * u1 * u2 + 2.0 * P12;
        J[5] = rho * u2 * u2 + 2.0 * P22;
        K[0] = rho * u2;
        K[1] = rho * u1 * u2 + P12;
        K[2] = rho * u2 * u2 + P22;
        K[3] = rho * u1 * u1 * u2 + u2 * P11 + 2.0 * u1 * P12;
        K[4] = rho * u1 * u2 * u2 + u1 * P22 + 2.0 * u2 * P12;
        K[5] = rho * u2 * u2 * u2 + 3.0 * u2 * P22;
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) F[m] = 0.5 * (sgn * a * J[m] + (1.0 + sgn * b) * K[m]);
}

// full flux f(q) / g(q) of (eq5-41) without the heat-flux terms
__device__ __forceinline__ void flux_full(const double q[6], int d, double F[6])
{
    const double rho = q[0], u1 = q[1] / rho, u2 = q[2] / rho;
    const double P11 = q[3] - q[1] * u1, P12 = q[4] - q[1] * u2, P22 = q[5] - q[2] * u2;
    if (d == 0) {
        F[0] = rho * u1;
        F[1] = rho * u1 * u1 + P11;
        F[2] = rho * u1 * u2 + P12;
        F[3] = rho * u1 * u1 * u1 + 3.0 * u1 * P11;
        F[4] = rho * u1 * u1 * u2 + u2 * P11 + 2.0 * u1 * P12;
        F[5] = rho * u1 * u2 * u2 + u1 * P22 + 2.0 * u2 * P12;
    } else {
        F[0] = rho * u2;
        F[1] = rho * u1 * u2 + P12;
        F[2] = rho * u2 * u2 + P22;
        F[3] = rho * u1 * u1 * u2 + u2 * P11 + 2.0 * u1 * P12;
        F[4] = rho * u1 * u2 * u2 + u1 * P22 + 2.0 * u2 * P12;
        F[5] = rho * u2 * u2 * u2 + 3.0 * u2 * P22;
    }
}

// R^{+-}_a of (twodim_wall_densities_1)
__device__ __forceinline__ double wall_R(double u, double Taa, double Tw, double sgn)
{
    return sqrt(Taa / Tw) * exp(-u * u / (2.0 * Taa)) +
           u * sqrt(MM_PI / (2.0 * Tw)) * (erf(u / sqrt(2.0 * Taa)) + sgn);
}

// Ghost Maxwellian (rho, u1, u2, T) beyond side s of a cell whose own state is
// (rho, u1, u2, T11 (x sides) or T22 (y sides)); wall density from zero net
// normal mass flux, inflow state fixed.
__device__ __forceinline__ void side_ghost(const Side &S, int s, double rho, double u1, double u2,
                                           double Tnn, double g[4])
{
    if (S.kind == BC_INFLOW) {
        g[0] = S.rho; g[1] = S.u1; g[2] = S.u2; g[3] = S.T;
        return;
    }
    const double sgn = (s == 0 || s == 2) ? -1.0 : 1.0;
    const double un = s < 2 ? u1 : u2;
    g[0] = rho * wall_R(un, Tnn, S.T_wall, sgn);
    g[1] = s < 2 ? 0.0 : S.u_wall;
    g[2] = s < 2 ? S.u_wall : 0.0;
    g[3] = S.T_wall;
}

__device__ __forceinline__ void ghost_q(const double g[4], double q[6])
{
    q[0] = g[0];
    q[1] = g[0] * g[1];
    q[2] = g[0] * g[2];
    q[3] = g[0] * g[1] * g[1] + g[0] * g[3];
    q[4] = g[0] * g[1] * g[2];
    q[5] = g[0] * g[2] * g[2] + g[0] * g[3];
}

__device__ __forceinline__ bool q_bad(const double q[6])
{
    const double rho = q[0];
    if (!(rho > 0.0)) return true;
    const double u1 = q[1] / rho, u2 = q[2] / rho;
    const double P11 = q[3] - q[1] * u1, P22 = q[5] - q[2] * u2, P12 = q[4] - q[1] * u2;
    if (!isfinite(u1) || !isfinite(u2) || !isfinite(P11) || !isfinite(P22) || !isfinite(P12)) return true;
    return !(P11 > 0.0) || !(P22 > 0.0);
}

} // namespace mm
