// mm_kernels2d.hip -- 2D2V ES-BGK micro-macro step on gfx950 (FP64 reference
// kernels: one workgroup per spatial cell for the phase-space pass, one thread
// per cell for the per-cell work).
//
// Paper: Rossmanith & Sar, arXiv:2509.21832, Sec. 5.3 (micro step) and
// Sec. 5.4 (macro step); walls of Sec. 6.3.
#include "mm_device.h"
#include "mm_launch.h"

namespace mm {

// ---------------------------------------------------------------------------
// per-cell preparation from Q^n

struct CellPrim {
    double rho, u1, u2, P11, P12, P22, p, T;
};

__device__ __forceinline__ CellPrim prim_of(const double *q)
{
    CellPrim c;
    c.rho = q[0];
    const double ir = 1.0 / q[0];   // one division per cell
    c.u1 = q[1] * ir;
    c.u2 = q[2] * ir;
    c.P11 = q[3] - q[1] * c.u1;
    c.P12 = q[4] - q[1] * c.u2;
    c.P22 = q[5] - q[2] * c.u2;
    c.p = 0.5 * (c.P11 + c.P22);
    c.T = c.p * ir;
    return c;
}

// neighbour cell along x (dir 0) or y (dir 1), `up` = +1 side; returns the cell
// index to read (the cell itself for extrapolation and open sides)
__device__ __forceinline__ int nbr_cell(const Params &P, int i, int j, int dir, int up)
{
    if (dir == 0) {
        if (up) return i < P.nx - 1 ? j * P.nx + i + 1 : (P.bc[1].kind == BC_PERIODIC ? j * P.nx : j * P.nx + i);
        return i > 0 ? j * P.nx + i - 1 : (P.bc[0].kind == BC_PERIODIC ? j * P.nx + P.nx - 1 : j * P.nx + i);
    }
    if (up) return j < P.ny - 1 ? (j + 1) * P.nx + i : (P.bc[3].kind == BC_PERIODIC ? i : j * P.nx + i);
    return j > 0 ? (j - 1) * P.nx + i : (P.bc[2].kind == BC_PERIODIC ? (P.ny - 1) * P.nx + i : j * P.nx + i);
}

__device__ __forceinline__ bool wall_cell(const Params &P, int i, int j)
{
    return (i == 0 && is_open(P.bc[0].kind)) || (i == P.nx - 1 && is_open(P.bc[1].kind)) ||
           (j == 0 && is_open(P.bc[2].kind)) || (j == P.ny - 1 && is_open(P.bc[3].kind));
}

// inverse of a symmetric positive definite 4x4 matrix (Cholesky); out packed by
// sym4.  The four diagonal factors are inverted once and the solves multiply.
__device__ __forceinline__ void spd_inverse4(const double A[4][4], double scale, double *out)
{
    double L[4][4] = {}, iL[4];
    for (int r = 0; r < 4; ++r) {
        for (int s = 0; s <= r; ++s) {
            double v = A[r][s];
            for (int t = 0; t < s; ++t) v -= L[r][t] * L[s][t];
            if (r == s) {
                L[r][r] = sqrt(v);
                iL[r] = 1.0 / L[r][r];
            } else {
                L[r][s] = v * iL[s];
            }
        }
    }
    // inverse columns: solve L L^T x = e_c
    double X[4][4];
    for (int col = 0; col < 4; ++col) {
        double y[4];
        for (int r = 0; r < 4; ++r) {
            double v = (r == col) ? 1.0 : 0.0;
            for (int t = 0; t < r; ++t) v -= L[r][t] * y[t];
            y[r] = v * iL[r];
        }
        for (int r = 3; r >= 0; --r) {
            double v = y[r];
            for (int t = r + 1; t < 4; ++t) v -= L[t][r] * X[t][col];
            X[r][col] = v * iL[r];
        }
    }
    for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b) out[sym4(a, b)] = scale * 0.5 * (X[a][b] + X[b][a]);
}

// S[q] = sum_k w_k^q exp(-w_k^2 i2T), q = 0..4, over the nodes w_k = w0 + (k + 1/2) h,
// k < n.  The Gaussian follows e(k+1) = e(k) r(k), r(k+1) = r(k) kappa (its
// exponent is quadratic in k) from one pair of exponentials at the first node:
// the range rule keeps every node's exponent within EXP_RANGE, so no value
// leaves the range of FP64, and the relative error grows like k^2 / 2 ulps
// (below 2e-13 of each moment's scale for 64 nodes, as small as restarting
// the recurrence every 8 nodes, which cost two exponentials per chunk).  Within
// a chunk of 8 nodes the sums run over the centred index t = k - 7/2 (exact
// constants): T_p = sum t^p e, and S_q gains sum_p C(q, p) wc^(q-p) h^p T_p with
// wc the chunk's centre.
__device__ inline void gauss_sums(double w0, double h, int n, double i2T, double S[5])
{
    const double kap = exp(-2.0 * h * h * i2T);
    const double h2 = h * h, h3 = h2 * h, h4 = h2 * h2;
    const double wf = w0 + 0.5 * h;
    double e = exp(-wf * wf * i2T), r = exp(-(2.0 * wf + h) * h * i2T);
    for (int k0 = 0; k0 < n; k0 += 8) {
        const double wb = w0 + (k0 + 0.5) * h;
        const int kn = n - k0 < 8 ? n - k0 : 8;
        double T[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < kn) {
                const double t = k - 3.5;
                T[0] += e;
                T[1] += t * e;
                T[2] += (t * t) * e;
                T[3] += (t * t * t) * e;
                T[4] += (t * t * t * t) * e;
                e *= r;
                r *= kap;
            }
        }
        const double wc = wb + 3.5 * h, wc2 = wc * wc, wc3 = wc2 * wc;
        S[0] += T[0];
        S[1] += wc * T[0] + h * T[1];
        S[2] += wc2 * T[0] + 2.0 * wc * h * T[1] + h2 * T[2];
        S[3] += wc3 * T[0] + 3.0 * wc2 * h * T[1] + 3.0 * wc * h2 * T[2] + h3 * T[3];
        S[4] += wc2 * wc2 * T[0] + 4.0 * wc3 * h * T[1] + 6.0 * wc2 * h2 * T[2] + 4.0 * wc * h3 * T[3] + h4 * T[4];
    }
}

// Four wavefronts per block of 64 cells, each assembling part of every cell's
// record (one cell per lane; the per-cell work is a long chain of dependent FP64
// operations: split four ways it is shorter, and four times as many wavefronts
// hide each other's latency):
//   wavefront 0: primitives, ES tensor and its Gaussian form, validity and range checks
//   wavefront 1: tau, relaxation weights, Maxwellian scalars, v2 Gram sums
//   wavefront 2: v1 Gram sums, the projection matrix (with wavefront 1's sums)
//   wavefront 3: central differences from the four neighbours, wall neighbour Maxwellians
// The records of the block's cells are assembled in LDS and written out together,
// so the stores are coalesced.
constexpr int PREP_CELLS = 64;

__global__ __launch_bounds__(4 * PREP_CELLS) void k_prep2d(const double *__restrict__ Q, double *__restrict__ rec,
                                                           double *__restrict__ wrec, int *__restrict__ flag,
                                                           int step, Params P)
{
    __shared__ double s_rec[PREP_CELLS * REC];
    __shared__ double s_s2[5][PREP_CELLS];
    const int ncell = P.nx * P.ny;
    const int c0 = blockIdx.x * PREP_CELLS;
    const int cl = threadIdx.x & 63;
    const int role = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = c0 + cl;
    double *R = s_rec + cl * REC;
    const bool discrete = P.proj_mode != PROJ_PAPER;
    if (c < ncell) {
        const int i = c % P.nx, j = c / P.nx;
        const CellPrim s = prim_of(Q + 6 * (size_t)c);
        const double iT = 1.0 / s.T, i2T = 0.5 * iT;   // 0.5 / T exactly as 1 / (2T)
        const double h = lk_step(P.nv1, P.nv2, P.dv2);
        if (role == 0) {
            // one reciprocal each of rho, 2 det and sqrt(det) instead of eight divisions
            const double nir = P.nu / s.rho;
            const double S11 = (1.0 - P.nu) * s.T + nir * s.P11;
            const double S12 = nir * s.P12;
            const double S22 = (1.0 - P.nu) * s.T + nir * s.P22;
            const double det = S11 * S22 - S12 * S12;
            if (!(s.rho > 0.0) || !(s.T > 0.0) || !(det > 0.0) || !(s.P11 > 0.0) || !(s.P22 > 0.0) ||
                !isfinite(s.u1) || !isfinite(s.u2) || !isfinite(s.P12))
                atomicMin(flag, step);
            R[R_RHO] = s.rho;
            R[R_U1] = s.u1;
            R[R_U2] = s.u2;
            R[R_T] = s.T;
            const double isd = 1.0 / sqrt(det), i2d = 0.5 / det;
            R[R_GPRE] = s.rho * isd * (0.5 / MM_PI);
            const double qa = S22 * i2d, qb = -S12 * i2d, qc = S11 * i2d;
            R[R_QA] = qa;
            R[R_QB] = qb;
            R[R_QC] = qc;
            R[R_LG] = log(s.T * isd);
            R[R_DA] = qa - i2T;
            R[R_DC] = qc - i2T;
            R[R_KG] = exp(-2.0 * qc * h * h);
            if (!exp_range_ok(P.v1_lo, P.dv1, P.nv1, P.v2_lo, P.dv2, P.nv2, s.u1, s.u2, i2T, qa, qb, qc))
                atomicMin(flag, step);
        } else if (role == 1) {
            for (int q = R_PM + 10; q < REC; ++q) R[q] = 0.0;    // unused tail of the record
            const double tau = tau_of(P, s.rho, s.p, s.T);
            // the reciprocals of T (above), tau, eps and eps + dt tau serve every quotient
            const double iw = 1.0 / (P.eps + P.dt * tau);
            R[R_RST] = sqrt(iT);
            R[R_MPRE] = s.rho * iT * (0.5 / MM_PI);
            R[R_I2T] = i2T;
            R[R_TAU] = tau;
            R[R_ITAU] = 1.0 / tau;
            R[R_IEPS] = 1.0 / P.eps;
            R[R_A] = P.eps * iw;
            R[R_B] = P.dt * tau * iw;
            R[R_IT] = iT;
            R[R_KM] = exp(-2.0 * h * h * i2T);
            // Gram_ab = dA sum phi_a phi_b M from separable 1D sums: M = c0 e1(k) e2(l)
            if (discrete) {
                double S2[5] = {0, 0, 0, 0, 0};
                gauss_sums(P.v2_lo - s.u2, P.dv2, P.nv2, i2T, S2);
                for (int q = 0; q < 5; ++q) s_s2[q][cl] = S2[q];
            }
        } else if (role == 3) {
            // central differences of u and T (eqn5-97, eqn5-97more) with boundary ghosts
            const CellPrim xm = prim_of(Q + 6 * (size_t)nbr_cell(P, i, j, 0, 0));
            const CellPrim xp = prim_of(Q + 6 * (size_t)nbr_cell(P, i, j, 0, 1));
            const CellPrim ym = prim_of(Q + 6 * (size_t)nbr_cell(P, i, j, 1, 0));
            const CellPrim yp = prim_of(Q + 6 * (size_t)nbr_cell(P, i, j, 1, 1));
            const double Tip = 0.5 * (xp.T + s.T), Tim = 0.5 * (xm.T + s.T);
            const double Tjp = 0.5 * (yp.T + s.T), Tjm = 0.5 * (ym.T + s.T);
            R[R_DTX] = (Tip - Tim) / P.dx;
            R[R_DTY] = (Tjp - Tjm) / P.dy;
            const double Dxu1 = 0.5 * (xp.u1 - xm.u1), Dxu2 = 0.5 * (xp.u2 - xm.u2);
            const double Dyu1 = 0.5 * (yp.u1 - ym.u1), Dyu2 = 0.5 * (yp.u2 - ym.u2);
            R[R_S11] = Dxu1 / P.dx - Dyu2 / P.dy;
            R[R_S12] = Dyu1 / P.dy + Dxu2 / P.dx;

            const bool wall = wall_cell(P, i, j);
            R[R_WALL] = wall ? 1.0 : 0.0;
            if (wall) {
                double *Wr = wrec + (size_t)c * WREC;
                const CellPrim *nb[4] = {&xm, &xp, &ym, &yp};
                for (int d = 0; d < 4; ++d) {
                    const int dir = d / 2, up = d % 2;
                    const bool inside = dir == 0 ? (up ? i < P.nx - 1 : i > 0) : (up ? j < P.ny - 1 : j > 0);
                    const int side = dir == 0 ? (up ? 1 : 0) : (up ? 3 : 2);
                    double g[4];
                    if (!inside && is_open(P.bc[side].kind)) {
                        side_ghost(P.bc[side], side, s.rho, s.u1, s.u2, side < 2 ? s.P11 / s.rho : s.P22 / s.rho, g);
                    } else {
                        g[0] = nb[d]->rho; g[1] = nb[d]->u1; g[2] = nb[d]->u2; g[3] = nb[d]->T;
                    }
                    Wr[4 * d + 0] = g[0] / (2.0 * MM_PI * g[3]);
                    Wr[4 * d + 1] = g[1];
                    Wr[4 * d + 2] = g[2];
                    Wr[4 * d + 3] = 1.0 / (2.0 * g[3]);
                    // the wall kernel follows these Maxwellians along the velocity nodes too
                    if (!exp_range_ok(P.v1_lo, P.dv1, P.nv1, P.v2_lo, P.dv2, P.nv2, g[1], g[2], Wr[4 * d + 3],
                                      Wr[4 * d + 3], 0.0, Wr[4 * d + 3]))
                        atomicMin(flag, step);
                }
            }
        }
    }
    // wavefront 2: the v1 sums, then (after wavefront 1's v2 sums are in LDS) the
    // projection matrix
    double S1[5] = {0, 0, 0, 0, 0};
    if (role == 2 && c < ncell && discrete) {
        const CellPrim s = prim_of(Q + 6 * (size_t)c);
        gauss_sums(P.v1_lo - s.u1, P.dv1, P.nv1, 1.0 / (2.0 * s.T), S1);
    }
    __syncthreads();
    const int ncopy = (ncell - c0 < PREP_CELLS ? ncell - c0 : PREP_CELLS) * REC;
    double *dst = rec + (size_t)c0 * REC;
    // while wavefront 2 forms the projection matrices, the other three write out
    // every other field of the block's records
    if (role != 2) {
        const int t0 = (role == 3 ? 2 : role) * PREP_CELLS + cl;
        for (int t = t0; t < ncopy; t += 3 * PREP_CELLS) {
            const int f = t % REC;
            if ((f < R_P0 || f >= R_P0 + 10) && (f < R_PM || f >= R_PM + 10)) dst[t] = s_rec[t];
        }
    }
    if (role == 2 && c < ncell) {
        const CellPrim s = prim_of(Q + 6 * (size_t)c);
        {
            // projection coefficients
            const double dA = P.dv1 * P.dv2;
            if (!discrete) {
                for (int a = 0; a < 4; ++a)
                    for (int b = a; b < 4; ++b) R[R_P0 + sym4(a, b)] = a == b ? dA / s.rho : 0.0;
            } else {
                double S2r[5];
                for (int q = 0; q < 5; ++q) S2r[q] = s_s2[q][cl];
                auto mm = [&](int p, int q) { return S1[p] * S2r[q]; };
                const double T = s.T, iT = 1.0 / T, irT = sqrt(iT), i2T = 0.5 * iT;
                const double c0 = dA * s.rho * (0.5 / MM_PI) * iT;
                double A[4][4];
                A[0][0] = c0 * mm(0, 0);
                A[0][1] = c0 * mm(1, 0) * irT;
                A[0][2] = c0 * mm(0, 1) * irT;
                A[0][3] = c0 * ((mm(2, 0) + mm(0, 2)) * i2T - mm(0, 0));
                A[1][1] = c0 * mm(2, 0) * iT;
                A[1][2] = c0 * mm(1, 1) * iT;
                A[1][3] = c0 * ((mm(3, 0) + mm(1, 2)) * i2T - mm(1, 0)) * irT;
                A[2][2] = c0 * mm(0, 2) * iT;
                A[2][3] = c0 * ((mm(2, 1) + mm(0, 3)) * i2T - mm(0, 1)) * irT;
                A[3][3] = c0 * ((mm(4, 0) + 2.0 * mm(2, 2) + mm(0, 4)) * (i2T * i2T) - (mm(2, 0) + mm(0, 2)) * iT + mm(0, 0));
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < a; ++b) A[a][b] = A[b][a];
                spd_inverse4(A, dA, R + R_P0);
            }
            // the same projection from raw moments: PM = T^t P0 T
            const double rsT = 1.0 / sqrt(s.T), i2T = 1.0 / (2.0 * s.T);
            const double Tm[4][4] = {{1.0, 0.0, 0.0, 0.0},
                                     {-rsT * s.u1, rsT, 0.0, 0.0},
                                     {-rsT * s.u2, 0.0, rsT, 0.0},
                                     {i2T * (s.u1 * s.u1 + s.u2 * s.u2) - 1.0, -2.0 * s.u1 * i2T,
                                      -2.0 * s.u2 * i2T, i2T}};
            double PT[4][4];
            for (int a = 0; a < 4; ++a)
                for (int q = 0; q < 4; ++q) {
                    double v = 0.0;
                    for (int b = 0; b < 4; ++b) v += R[R_P0 + sym4(a, b)] * Tm[b][q];
                    PT[a][q] = v;
                }
            for (int a = 0; a < 4; ++a)
                for (int q = a; q < 4; ++q) {
                    double v = 0.0;
                    for (int b = 0; b < 4; ++b) v += Tm[b][a] * PT[b][q];
                    R[R_PM + sym4(a, q)] = v;
                }
        }
    }
    __syncthreads();
    // then the two matrices (10 packed entries each) of every cell
    const int nmat = ncopy / REC * 20;
    for (int t = threadIdx.x; t < nmat; t += 4 * PREP_CELLS) {
        const int cc = t / 20, f = t % 20, q = cc * REC + (f < 10 ? R_P0 + f : R_PM + f - 10);
        dst[q] = s_rec[q];
    }
}

// ---------------------------------------------------------------------------
// phase-space pass, reference form: one workgroup per cell

__device__ __forceinline__ void proj_coef(const double *R, const double s[4], double A[4])
{
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) v += R[R_P0 + sym4(a, b)] * s[b];
        A[a] = v;
    }
}

// x-transport sub-step (micro-2D-split-1): G -> G*
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_micro_x2d(const double *__restrict__ G, double *__restrict__ Gs,
                                                      const double *__restrict__ rec, Params P)
{
    __shared__ double lds[NW * 4];
    const int c = blockIdx.x, i = c % P.nx;
    const double *R = rec + (size_t)c * REC;
    const double u1 = R[R_U1], u2 = R[R_U2], rsT = R[R_RST], i2T = R[R_I2T], mpre = R[R_MPRE];
    const size_t nv = P.nv;
    const double *Gc = G + (size_t)c * nv;
    const double *Gm, *Gp;
    if (i > 0) Gm = Gc - nv;
    else if (P.bc[0].kind == BC_PERIODIC) Gm = Gc + (size_t)(P.nx - 1) * nv;
    else Gm = is_open(P.bc[0].kind) ? nullptr : Gc;
    if (i < P.nx - 1) Gp = Gc + nv;
    else if (P.bc[1].kind == BC_PERIODIC) Gp = Gc - (size_t)(P.nx - 1) * nv;
    else Gp = is_open(P.bc[1].kind) ? nullptr : Gc;

    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < P.nv; p += 64 * NW) {
        const int k = p % P.nv1, l = p / P.nv1;
        const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
        const double gc = Gc[p], gm = Gm ? Gm[p] : 0.0, gp = Gp ? Gp[p] : 0.0;
        const double Z = fmin(0.0, v1) * ((gp - gc) / P.dx) + fmax(0.0, v1) * ((gc - gm) / P.dx);
        const double w1 = v1 - u1, w2 = v2 - u2;
        s[0] += Z;
        s[1] += w1 * rsT * Z;
        s[2] += w2 * rsT * Z;
        s[3] += ((w1 * w1 + w2 * w2) * i2T - 1.0) * Z;
    }
    block_sum<4, NW>(s, lds);
    double A[4];
    proj_coef(R, s, A);
    for (int p = threadIdx.x; p < P.nv; p += 64 * NW) {
        const int k = p % P.nv1, l = p / P.nv1;
        const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
        const double gc = Gc[p], gm = Gm ? Gm[p] : 0.0, gp = Gp ? Gp[p] : 0.0;
        const double Z = fmin(0.0, v1) * ((gp - gc) / P.dx) + fmax(0.0, v1) * ((gc - gm) / P.dx);
        const double w1 = v1 - u1, w2 = v2 - u2, r2 = w1 * w1 + w2 * w2;
        const double M = mpre * exp(-r2 * i2T);
        const double Zh = (A[0] + A[1] * (w1 * rsT) + A[2] * (w2 * rsT) + A[3] * (r2 * i2T - 1.0)) * M;
        Gs[(size_t)c * nv + p] = gc + P.dt * (Zh - Z);
    }
}

// Maxwellian from (rho / (2 pi T), u1, u2, 1 / (2T))
__device__ __forceinline__ double maxw(double pre, double u1, double u2, double i2T, double v1, double v2)
{
    const double w1 = v1 - u1, w2 = v2 - u2;
    return pre * exp(-(w1 * w1 + w2 * w2) * i2T);
}

// y-transport (micro-2D-split-2), G-hat (eqn5-97 / wall form), relaxation
// (eqn5-98) and the heat-flux tensor (eqn5-99): G* -> G^{n+1}, H^{n+1}
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_micro_y2d(const double *__restrict__ Gs, double *__restrict__ Gn,
                                                      double *__restrict__ H, const double *__restrict__ rec,
                                                      const double *__restrict__ wrec, Params P)
{
    __shared__ double lds[NW * 12];
    const int c = blockIdx.x, j = c / P.nx;
    const double *R = rec + (size_t)c * REC;
    const double u1 = R[R_U1], u2 = R[R_U2], rsT = R[R_RST], i2T = R[R_I2T], mpre = R[R_MPRE];
    const double gpre = R[R_GPRE], qa = R[R_QA], qb = R[R_QB], qc = R[R_QC], ieps = R[R_IEPS];
    const double itau = R[R_ITAU], s11 = R[R_S11], s12 = R[R_S12], dTx = R[R_DTX], dTy = R[R_DTY];
    const double T = R[R_T];
    const bool wall = R[R_WALL] != 0.0;
    const bool discrete = P.proj_mode == PROJ_DISCRETE;
    const bool es_on = !wall || P.wall_es_term;
    double nbm[16];
    if (wall)
        for (int t = 0; t < 16; ++t) nbm[t] = wrec[(size_t)c * WREC + t];
    const size_t nv = P.nv, row = (size_t)P.nx * nv;
    const double *Gc = Gs + (size_t)c * nv;
    const double *Gm, *Gp;
    if (j > 0) Gm = Gc - row;
    else if (P.bc[2].kind == BC_PERIODIC) Gm = Gc + (size_t)(P.ny - 1) * row;
    else Gm = is_open(P.bc[2].kind) ? nullptr : Gc;
    if (j < P.ny - 1) Gp = Gc + row;
    else if (P.bc[3].kind == BC_PERIODIC) Gp = Gc - (size_t)(P.ny - 1) * row;
    else Gp = is_open(P.bc[3].kind) ? nullptr : Gc;

    auto point = [&](int p, double &Z, double &M, double &mup, double &base, double &w1, double &w2, double &gc) {
        const int k = p % P.nv1, l = p / P.nv1;
        const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
        gc = Gc[p];
        const double gm = Gm ? Gm[p] : 0.0, gp = Gp ? Gp[p] : 0.0;
        Z = fmin(0.0, v2) * ((gp - gc) / P.dy) + fmax(0.0, v2) * ((gc - gm) / P.dy);
        w1 = v1 - u1;
        w2 = v2 - u2;
        const double r2 = w1 * w1 + w2 * w2;
        M = mpre * exp(-r2 * i2T);
        const double es = es_on ? (gpre * exp(-(qa * w1 * w1 + 2.0 * qb * w1 * w2 + qc * w2 * w2)) - M) * ieps : 0.0;
        if (wall) {
            const double Mxm = maxw(nbm[0], nbm[1], nbm[2], nbm[3], v1, v2);
            const double Mxp = maxw(nbm[4], nbm[5], nbm[6], nbm[7], v1, v2);
            const double Mym = maxw(nbm[8], nbm[9], nbm[10], nbm[11], v1, v2);
            const double Myp = maxw(nbm[12], nbm[13], nbm[14], nbm[15], v1, v2);
            mup = fmin(0.0, v1) * ((Mxp - M) / P.dx) + fmax(0.0, v1) * ((M - Mxm) / P.dx) +
                  fmin(0.0, v2) * ((Myp - M) / P.dy) + fmax(0.0, v2) * ((M - Mym) / P.dy);
            base = es;
        } else {
            mup = 0.0;
            const double Bs = (s11 * (w1 * w1 - w2 * w2) + 2.0 * s12 * w1 * w2) / (2.0 * T);
            const double CgT = ((r2 / (2.0 * T) - 2.0) / T) * (w1 * dTx + w2 * dTy);
            base = -itau * (Bs + CgT) * M + es;
        }
    };

    double s[12];
#pragma unroll
    for (int n = 0; n < 12; ++n) s[n] = 0.0;
    for (int p = threadIdx.x; p < P.nv; p += 64 * NW) {
        double Z, M, mup, base, w1, w2, gc;
        point(p, Z, M, mup, base, w1, w2, gc);
        const double f[4] = {1.0, w1 * rsT, w2 * rsT, (w1 * w1 + w2 * w2) * i2T - 1.0};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            s[a] += f[a] * Z;
            s[4 + a] += f[a] * mup;
            s[8 + a] += f[a] * base;
        }
    }
    block_sum<12, NW>(s, lds);
    double AZ[4], AM[4], AB[4];
    proj_coef(R, s, AZ);
    proj_coef(R, s + 4, AM);
    proj_coef(R, s + 8, AB);
    if (!discrete)
        for (int a = 0; a < 4; ++a) AB[a] = 0.0;
    const double ra = R[R_A], rb = R[R_B];
    double h[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < P.nv; p += 64 * NW) {
        double Z, M, mup, base, w1, w2, gc;
        point(p, Z, M, mup, base, w1, w2, gc);
        const double f1 = w1 * rsT, f2 = w2 * rsT, f3 = (w1 * w1 + w2 * w2) * i2T - 1.0;
        const double Zh = (AZ[0] + AZ[1] * f1 + AZ[2] * f2 + AZ[3] * f3) * M;
        const double gss = gc + P.dt * (Zh - Z);
        const double PM = (AM[0] + AM[1] * f1 + AM[2] * f2 + AM[3] * f3) * M;
        const double PB = (AB[0] + AB[1] * f1 + AB[2] * f2 + AB[3] * f3) * M;
        const double gh = -itau * (mup - PM) + (base - PB);
        const double gn = ra * gss + rb * gh;
        Gn[(size_t)c * nv + p] = gn;
        h[0] += w1 * w1 * w1 * gn;
        h[1] += w1 * w1 * w2 * gn;
        h[2] += w1 * w2 * w2 * gn;
        h[3] += w2 * w2 * w2 * gn;
    }
    block_sum<4, NW>(h, lds);
    if (threadIdx.x == 0) {
        const double f = P.eps * P.dv1 * P.dv2;
        for (int a = 0; a < 4; ++a) H[(size_t)c * 4 + a] = f * h[a];
    }
}

// ---------------------------------------------------------------------------
// macro sweeps (eqn5-103) with the collision half steps fused in

// face flux and heat-flux face value between the cells at positions m-1 and m
// along a line; qlo / qhi are the collided states of those cells.
__device__ __forceinline__ void interior_face(const double qlo[6], const double qhi[6], int d, double F[6])
{
    double fp[6], fm[6];
    kfvs_half(qlo, d, 1.0, fp);
    kfvs_half(qhi, d, -1.0, fm);
#pragma unroll
    for (int m = 0; m < 6; ++m) F[m] = fp[m] + fm[m];
}

// boundary face of side `side` next to the edge cell with collided state qe
__device__ __forceinline__ void boundary_face(const Params &P, int side, const double qe[6], const double qwrap[6],
                                              int d, double F[6])
{
    const int kind = P.bc[side].kind;
    const bool low = (side == 0 || side == 2);
    if (kind == BC_EXTRAP) {
        flux_full(qe, d, F);
    } else if (kind == BC_PERIODIC) {
        if (low) interior_face(qwrap, qe, d, F);
        else interior_face(qe, qwrap, d, F);
    } else {
        const double rho = qe[0], u1 = qe[1] / rho, u2 = qe[2] / rho;
        const double Pnn = d == 0 ? qe[3] - qe[1] * u1 : qe[5] - qe[2] * u2;
        double g[4], qg[6];
        side_ghost(P.bc[side], side, rho, u1, u2, Pnn / rho, g);
        ghost_q(g, qg);
        if (low) interior_face(qg, qe, d, F);
        else interior_face(qe, qg, d, F);
    }
}

__device__ __forceinline__ void load_q(const double *Q, int c, double q[6])
{
#pragma unroll
    for (int m = 0; m < 6; ++m) q[m] = Q[6 * (size_t)c + m];
}

// dir 0: Q^n -> (collision half) Q* -> KFVS x -> Q**;  dir 1: Q** -> KFVS y -> Q*** -> (collision half) Q^{n+1}
// Four lanes per cell, one half flux each (the erf / exp of the half-space
// integrals dominate): lane 0 F+ of the low neighbour, lane 1 F- of the cell
// (the low face), lane 2 F+ of the cell, lane 3 F- of the high neighbour (the
// high face).  A boundary face is computed whole by lane 0 or 3 (the other
// lane of the face adds zero).  Lane 1 combines the faces and writes the cell.
template <int DIR>
__global__ __launch_bounds__(256) void k_macro2d(const double *__restrict__ Qin, const double *__restrict__ H,
                                                 double *__restrict__ Qout, int *__restrict__ flag, int step,
                                                 Params P, const double *__restrict__ msrc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = t >> 2, role = t & 3;
    if (c >= P.nx * P.ny) return;     // whole groups of four
    const int i = c % P.nx, j = c / P.nx;
    const int n = DIR == 0 ? P.nx : P.ny, pos = DIR == 0 ? i : j;
    const int stride = DIR == 0 ? 1 : P.nx;
    const int slo = DIR == 0 ? 0 : 2, shi = DIR == 0 ? 1 : 3;
    const double h = DIR == 0 ? P.dx : P.dy;
    const int hoff = DIR == 0 ? 0 : 1;
    const int cl = pos > 0 ? c - stride : c + (n - 1) * stride;      // periodic wrap when at the low edge
    const int cr = pos < n - 1 ? c + stride : c - (n - 1) * stride;
    const bool low_face = role < 2;
    const int side = low_face ? slo : shi;
    const bool at_bc = low_face ? pos == 0 : pos == n - 1;
    const bool whole = at_bc && P.bc[side].kind != BC_PERIODIC;      // a boundary face, not a wrap
    double r[6];
    if (whole) {
        if (role == 0 || role == 3) {
            double qc[6], qw[6];
            load_q(Qin, c, qc);
            load_q(Qin, role == 0 ? cl : cr, qw);
            if (DIR == 0) collide(P, qc);
            boundary_face(P, side, qc, qw, DIR, r);
        } else {
#pragma unroll
            for (int m = 0; m < 6; ++m) r[m] = 0.0;
        }
    } else {
        double q[6];
        load_q(Qin, role == 0 ? cl : role == 3 ? cr : c, q);
        if (DIR == 0) collide(P, q);
        kfvs_half(q, DIR, (role == 0 || role == 2) ? 1.0 : -1.0, r);
    }
    // faces: F_low = r(lane 0) + r(lane 1), F_high = r(lane 2) + r(lane 3)
    const int g0 = threadIdx.x & ~3;
    double FL[6], FR[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const double a0 = __shfl(r[m], g0, 64), a1 = __shfl(r[m], g0 + 1, 64);
        const double a2 = __shfl(r[m], g0 + 2, 64), a3 = __shfl(r[m], g0 + 3, 64);
        FL[m] = a0 + a1;
        FR[m] = a2 + a3;
    }
    if (role != 1) return;
    double qc[6];
    load_q(Qin, c, qc);
    if (DIR == 0) collide(P, qc);
    double HL[3], HR[3];
    if (pos > 0) {
        for (int a = 0; a < 3; ++a) HL[a] = 0.5 * (H[4 * (size_t)c + hoff + a] + H[4 * (size_t)cl + hoff + a]);
    } else {
        const int kind = P.bc[slo].kind;
        for (int a = 0; a < 3; ++a) {
            const double hc = H[4 * (size_t)c + hoff + a];
            HL[a] = kind == BC_EXTRAP ? hc : kind == BC_PERIODIC ? 0.5 * (hc + H[4 * (size_t)cl + hoff + a]) : 0.5 * hc;
        }
    }
    if (pos < n - 1) {
        for (int a = 0; a < 3; ++a) HR[a] = 0.5 * (H[4 * (size_t)cr + hoff + a] + H[4 * (size_t)c + hoff + a]);
    } else {
        const int kind = P.bc[shi].kind;
        for (int a = 0; a < 3; ++a) {
            const double hc = H[4 * (size_t)c + hoff + a];
            HR[a] = kind == BC_EXTRAP ? hc : kind == BC_PERIODIC ? 0.5 * (H[4 * (size_t)cr + hoff + a] + hc) : 0.5 * hc;
        }
    }
    double qo[6];
    for (int m = 0; m < 6; ++m) qo[m] = qc[m] - P.dt / h * (FR[m] - FL[m]);
    for (int a = 0; a < 3; ++a) qo[3 + a] -= P.dt / h * (HR[a] - HL[a]);
    if (DIR == 1) {
        if (msrc)
            for (int m = 0; m < 6; ++m) qo[m] += P.dt * msrc[6 * (size_t)c + m];
        collide(P, qo);
        if (q_bad(qo)) atomicMin(flag, step + 1);
    }
    for (int m = 0; m < 6; ++m) Qout[6 * (size_t)c + m] = qo[m];
}

// The same sweep with one workgroup per line of cells along the sweep (a row
// for dir 0, a column for dir 1; lines of at most MACRO_LINE cells).  Each cell
// is collided and its two half fluxes are formed once, F+ by an even lane and
// F- by the odd lane next to it, into LDS; the faces are then F+ (low cell) +
// F- (high cell), the wrap for a periodic side, or the boundary face of the
// edge cell, and the even lane updates the cell.  The heat-flux values a cell
// needs are loaded before the flux work so their latency overlaps it.  (The
// four-lane form above repeats the collision and the half fluxes of a cell up
// to five times, which made it bound by FP64 arithmetic.)
constexpr int MACRO_LINE = 512;   // 48 KB of LDS per workgroup at most
constexpr int MACRO_THREADS = 512;

template <int DIR>
__global__ __launch_bounds__(MACRO_THREADS) void k_macro_line(const double *__restrict__ Qin,
                                                              const double *__restrict__ H,
                                                              double *__restrict__ Qout, int *__restrict__ flag,
                                                              int step, Params P, const double *__restrict__ msrc)
{
    extern __shared__ double s_f[];   // [2][n][6]: F+ and F- of every cell of the line
    const int n = DIR == 0 ? P.nx : P.ny;
    const int nline = DIR == 0 ? P.ny : P.nx;
    // dispatch puts workgroup b on XCD b mod 8: neighbouring lines share an XCD
    const int per = (nline + 7) / 8;
    const int line = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (line >= nline) return;
    const int stride = DIR == 0 ? 1 : P.nx;
    const int base = DIR == 0 ? line * P.nx : line;
    const int slo = DIR == 0 ? 0 : 2, shi = DIR == 0 ? 1 : 3;
    const double h = DIR == 0 ? P.dx : P.dy;
    const int hoff = DIR == 0 ? 0 : 1;
    const bool odd = (threadIdx.x & 1) != 0;
    double *Fp = s_f, *Fm = s_f + 6 * n;
    constexpr int CPT = MACRO_LINE / (MACRO_THREADS / 2);   // cells per lane pair
    double qs[CPT][6], hc[CPT][3], hl[CPT][3], hr[CPT][3];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int pos = (threadIdx.x >> 1) + (MACRO_THREADS / 2) * u;
        if (pos >= n) break;
        const int c = base + pos * stride;
        const int cl = pos > 0 ? c - stride : c + (n - 1) * stride;
        const int cr = pos < n - 1 ? c + stride : c - (n - 1) * stride;
        load_q(Qin, c, qs[u]);
        if (!odd) {
            for (int a = 0; a < 3; ++a) {
                hc[u][a] = H[4 * (size_t)c + hoff + a];
                hl[u][a] = H[4 * (size_t)cl + hoff + a];
                hr[u][a] = H[4 * (size_t)cr + hoff + a];
            }
        }
        if (DIR == 0) collide(P, qs[u]);
        double F[6];
        kfvs_half(qs[u], DIR, odd ? -1.0 : 1.0, F);
        double *dst = odd ? Fm : Fp;
#pragma unroll
        for (int m = 0; m < 6; ++m) dst[6 * pos + m] = F[m];
    }
    __syncthreads();
    if (odd) return;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int pos = (threadIdx.x >> 1) + (MACRO_THREADS / 2) * u;
        if (pos >= n) break;
        const int c = base + pos * stride;
        const double *qc = qs[u];
        double FL[6], FR[6];
        if (pos > 0) {
            for (int m = 0; m < 6; ++m) FL[m] = Fp[6 * (pos - 1) + m] + Fm[6 * pos + m];
        } else if (P.bc[slo].kind == BC_PERIODIC) {
            for (int m = 0; m < 6; ++m) FL[m] = Fp[6 * (n - 1) + m] + Fm[m];
        } else {
            boundary_face(P, slo, qc, qc, DIR, FL);
        }
        if (pos < n - 1) {
            for (int m = 0; m < 6; ++m) FR[m] = Fp[6 * pos + m] + Fm[6 * (pos + 1) + m];
        } else if (P.bc[shi].kind == BC_PERIODIC) {
            for (int m = 0; m < 6; ++m) FR[m] = Fp[6 * (n - 1) + m] + Fm[m];
        } else {
            boundary_face(P, shi, qc, qc, DIR, FR);
        }
        double HL[3], HR[3];
        if (pos > 0) {
            for (int a = 0; a < 3; ++a) HL[a] = 0.5 * (hc[u][a] + hl[u][a]);
        } else {
            const int kind = P.bc[slo].kind;
            for (int a = 0; a < 3; ++a)
                HL[a] = kind == BC_EXTRAP ? hc[u][a] : kind == BC_PERIODIC ? 0.5 * (hc[u][a] + hl[u][a]) : 0.5 * hc[u][a];
        }
        if (pos < n - 1) {
            for (int a = 0; a < 3; ++a) HR[a] = 0.5 * (hr[u][a] + hc[u][a]);
        } else {
            const int kind = P.bc[shi].kind;
            for (int a = 0; a < 3; ++a)
                HR[a] = kind == BC_EXTRAP ? hc[u][a] : kind == BC_PERIODIC ? 0.5 * (hr[u][a] + hc[u][a]) : 0.5 * hc[u][a];
        }
        double qo[6];
        for (int m = 0; m < 6; ++m) qo[m] = qc[m] - P.dt / h * (FR[m] - FL[m]);
        for (int a = 0; a < 3; ++a) qo[3 + a] -= P.dt / h * (HR[a] - HL[a]);
        if (DIR == 1) {
            if (msrc)
                for (int m = 0; m < 6; ++m) qo[m] += P.dt * msrc[6 * (size_t)c + m];
            collide(P, qo);
            if (q_bad(qo)) atomicMin(flag, step + 1);
        }
        for (int m = 0; m < 6; ++m) Qout[6 * (size_t)c + m] = qo[m];
    }
}

// g-moments for diagnostics: dv sum (1, v1, v2, |v|^2/2) G and
// eps dv sum ((w1^2 - w2^2)/2, w1 w2, |w|^2/2) G per cell
template <typename TG>
__global__ __launch_bounds__(256) void k_gmom2d(const TG *__restrict__ G, const double *__restrict__ rec,
                                                double *__restrict__ out, Params P)
{
    __shared__ double lds[4 * 7];
    const int c = blockIdx.x;
    const double u1 = rec[(size_t)c * REC + R_U1], u2 = rec[(size_t)c * REC + R_U2];
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < P.nv; p += 256) {
        const int k = p % P.nv1, l = p / P.nv1;
        const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
        const double g = (double)G[(size_t)c * P.nv + p];
        const double w1 = v1 - u1, w2 = v2 - u2;
        s[0] += g;
        s[1] += v1 * g;
        s[2] += v2 * g;
        s[3] += 0.5 * (v1 * v1 + v2 * v2) * g;
        s[4] += 0.5 * (w1 * w1 - w2 * w2) * g;
        s[5] += w1 * w2 * g;
        s[6] += 0.5 * (w1 * w1 + w2 * w2) * g;
    }
    block_sum<7, 4>(s, lds);
    if (threadIdx.x == 0) {
        const double dA = P.dv1 * P.dv2;
        for (int a = 0; a < 4; ++a) out[7 * (size_t)c + a] = dA * s[a];
        for (int a = 4; a < 7; ++a) out[7 * (size_t)c + a] = P.eps * dA * s[a];
    }
}

// ---------------------------------------------------------------------------
// wall-adjacent cells after a fused pass: Gn holds G** there.  This kernel
// applies the wall form of G-hat (Sec. 6.3: -(1/tau)(I - Pi)[upwind v.grad M
// with ghost Maxwellians] + (G - M)/eps), the relaxation (eqn5-98) and H
// (eqn5-99), in FP64 for both storage types.  One workgroup per cell of the
// boundary ring; cells that are not wall cells return at once.


// One workgroup per wall-adjacent cell.  The cell's Maxwellian and the four
// neighbour (ghost) Maxwellians are separable: 1D factors of each go to LDS
// tables (5 (nv1 + nv2) exponentials per cell instead of 5 nv).  The first
// pass keeps the upwind term and the ES term of every node in LDS for the second.
constexpr int WALL_MAXV = 64;      // nv1, nv2 of the fused pass
constexpr int WALL_MAXNV = 2304;   // nv of the fused pass

template <typename TS>
__global__ __launch_bounds__(256) void k_wall_relax2d(TS *__restrict__ Gn, double *__restrict__ H,
                                                      const double *__restrict__ rec,
                                                      const double *__restrict__ wrec, Params P)
{
    __shared__ double lds[4 * 8];
    __shared__ double e1[5][WALL_MAXV], e2[5][WALL_MAXV];   // 0: the cell; 1..4: x-, x+, y-, y+ neighbours
    __shared__ double s_mup[WALL_MAXNV], s_es[WALL_MAXNV];
    int i, j;
    ring_cell(P, blockIdx.x, i, j);
    const size_t c = (size_t)j * P.nx + i;
    const double *R = rec + c * REC;
    if (R[R_WALL] == 0.0) return;
    const double u1 = R[R_U1], u2 = R[R_U2], rsT = R[R_RST], i2T = R[R_I2T], mpre = R[R_MPRE];
    const double dA = R[R_DA], dB = R[R_QB], dC = R[R_DC], lg = R[R_LG], ieps = R[R_IEPS], itau = R[R_ITAU];
    const bool es_on = P.wall_es_term != 0, discrete = P.proj_mode == PROJ_DISCRETE;
    const double *nb = wrec + c * WREC;     // per neighbour: (rho / (2 pi T), u1, u2, 1 / (2T))
    const int n12 = P.nv1 + P.nv2;
    for (int t = threadIdx.x; t < 5 * n12; t += 256) {
        const int d = t / n12, q = t - d * n12;
        const double cu1 = d ? nb[4 * (d - 1) + 1] : u1, cu2 = d ? nb[4 * (d - 1) + 2] : u2;
        const double ci2T = d ? nb[4 * (d - 1) + 3] : i2T;
        if (q < P.nv1) {
            const double a = P.v1_lo + (q + 0.5) * P.dv1 - cu1;
            e1[d][q] = exp(-a * a * ci2T);
        } else {
            const double a = P.v2_lo + (q - P.nv1 + 0.5) * P.dv2 - cu2;
            e2[d][q - P.nv1] = exp(-a * a * ci2T);
        }
    }
    __syncthreads();
    const double pre0 = nb[0], pre1 = nb[4], pre2 = nb[8], pre3 = nb[12];
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int p = threadIdx.x; p < P.nv; p += 256) {
        const int k = p % P.nv1, l = p / P.nv1;
        const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
        const double w1 = v1 - u1, w2 = v2 - u2;
        const double M = mpre * e1[0][k] * e2[0][l];
        const double es = es_on ? M * expm1(lg - (dA * w1 * w1 + 2.0 * dB * w1 * w2 + dC * w2 * w2)) * ieps : 0.0;
        const double M0 = pre0 * e1[1][k] * e2[1][l], M1 = pre1 * e1[2][k] * e2[2][l];
        const double M2 = pre2 * e1[3][k] * e2[3][l], M3 = pre3 * e1[4][k] * e2[4][l];
        const double mup = (fmin(v1, 0.0) * (M1 - M) + fmax(v1, 0.0) * (M - M0)) / P.dx +
                           (fmin(v2, 0.0) * (M3 - M) + fmax(v2, 0.0) * (M - M2)) / P.dy;
        s_mup[p] = mup;
        s_es[p] = es;
        const double f1 = w1 * rsT, f2 = w2 * rsT, f3 = (w1 * w1 + w2 * w2) * i2T - 1.0;
        s[0] += mup;
        s[1] += f1 * mup;
        s[2] += f2 * mup;
        s[3] += f3 * mup;
        s[4] += es;
        s[5] += f1 * es;
        s[6] += f2 * es;
        s[7] += f3 * es;
    }
    block_sum<8, 4>(s, lds);     // its barriers also publish s_mup, s_es
    double AM[4], AE[4];
    proj_coef(R, s, AM);
    proj_coef(R, s + 4, AE);
    if (!discrete)
        for (int a = 0; a < 4; ++a) AE[a] = 0.0;
    const double ra = R[R_A], rb = R[R_B];
    TS *g = Gn + c * (size_t)P.nv;
    double h[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int p = threadIdx.x; p < P.nv; p += 256) {
        const int k = p % P.nv1, l = p / P.nv1;
        const double w1 = P.v1_lo + (k + 0.5) * P.dv1 - u1, w2 = P.v2_lo + (l + 0.5) * P.dv2 - u2;
        const double M = mpre * e1[0][k] * e2[0][l];
        const double f1 = w1 * rsT, f2 = w2 * rsT, f3 = (w1 * w1 + w2 * w2) * i2T - 1.0;
        const double PM = (AM[0] + AM[1] * f1 + AM[2] * f2 + AM[3] * f3) * M;
        const double PE = (AE[0] + AE[1] * f1 + AE[2] * f2 + AE[3] * f3) * M;
        const double gh = -itau * (s_mup[p] - PM) + (s_es[p] - PE);
        const TS gn = (TS)(ra * (double)g[p] + rb * gh);
        g[p] = gn;
        const double gv = (double)gn;
        h[0] += w1 * w1 * w1 * gv;
        h[1] += w1 * w1 * w2 * gv;
        h[2] += w1 * w2 * w2 * gv;
        h[3] += w2 * w2 * w2 * gv;
    }
    block_sum<4, 4>(h, lds);
    if (threadIdx.x == 0) {
        const double f = P.eps * P.dv1 * P.dv2;
        for (int a = 0; a < 4; ++a) H[c * 4 + a] = f * h[a];
    }
}

// ---------------------------------------------------------------------------
// launchers

void launch_prep2d(const double *Q, double *rec, double *wrec, int *flag, int step, const Params &P, hipStream_t st)
{
    const int n = P.nx * P.ny;
    hipLaunchKernelGGL(k_prep2d, dim3((n + PREP_CELLS - 1) / PREP_CELLS), dim3(4 * PREP_CELLS), 0, st, Q, rec, wrec,
                       flag, step, P);
}

void launch_micro_ref2d(const double *G, double *Gs, double *Gn, double *H, const double *rec, const double *wrec,
                        const Params &P, hipStream_t st)
{
    const int n = P.nx * P.ny;
    hipLaunchKernelGGL(k_micro_x2d<4>, dim3(n), dim3(256), 0, st, G, Gs, rec, P);
    hipLaunchKernelGGL(k_micro_y2d<4>, dim3(n), dim3(256), 0, st, Gs, Gn, H, rec, wrec, P);
}

void launch_macro2d(double *Q, double *Qs, const double *H, int *flag, int step, const Params &P, hipStream_t st,
                    const double *msrc)
{
    const int n = P.nx * P.ny;
    // one workgroup per line where a line fits MACRO_LINE cells, else four lanes per cell
    const auto line_grid = [](int nline) { return dim3(((nline + 7) / 8) * 8); };
    if (P.nx <= MACRO_LINE)
        hipLaunchKernelGGL(k_macro_line<0>, line_grid(P.ny), dim3(MACRO_THREADS), 12 * sizeof(double) * P.nx, st,
                           Q, H, Qs, flag, step, P, nullptr);
    else
        hipLaunchKernelGGL(k_macro2d<0>, dim3((4 * n + 255) / 256), dim3(256), 0, st, Q, H, Qs, flag, step, P,
                           nullptr);
    if (P.ny <= MACRO_LINE)
        hipLaunchKernelGGL(k_macro_line<1>, line_grid(P.nx), dim3(MACRO_THREADS), 12 * sizeof(double) * P.ny, st,
                           Qs, H, Q, flag, step, P, msrc);
    else
        hipLaunchKernelGGL(k_macro2d<1>, dim3((4 * n + 255) / 256), dim3(256), 0, st, Qs, H, Q, flag, step, P,
                           msrc);
}

void launch_wall_relax2d(void *Gn, int g_bytes, double *H, const double *rec, const double *wrec, const Params &P,
                         hipStream_t st)
{
    bool any = false;
    for (int s = 0; s < 4; ++s) any = any || is_open(P.bc[s].kind);
    if (!any) return;
    if (launch_wall_lk2d(Gn, g_bytes, H, rec, wrec, P, st)) return;
    const int n = 2 * P.nx + 2 * (P.ny - 2);
    if (P.nv1 > WALL_MAXV || P.nv2 > WALL_MAXV || P.nv > WALL_MAXNV) return;   // not a fused-pass shape
    if (g_bytes == 8)
        hipLaunchKernelGGL(k_wall_relax2d<double>, dim3(n), dim3(256), 0, st, (double *)Gn, H, rec, wrec, P);
    else
        hipLaunchKernelGGL(k_wall_relax2d<float>, dim3(n), dim3(256), 0, st, (float *)Gn, H, rec, wrec, P);
}

void launch_gmom2d(const void *G, int g_bytes, const double *rec, double *out, const Params &P, hipStream_t st)
{
    const int n = P.nx * P.ny;
    if (g_bytes == 8)
        hipLaunchKernelGGL(k_gmom2d<double>, dim3(n), dim3(256), 0, st, (const double *)G, rec, out, P);
    else
        hipLaunchKernelGGL(k_gmom2d<float>, dim3(n), dim3(256), 0, st, (const float *)G, rec, out, P);
}

} // namespace mm
