// mm_internal.h -- device-side parameters and cell-record layout shared by the
// library's HIP translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MM_PI 3.14159265358979323846

namespace mm {

// boundary kinds (same values as the ABI)
enum { BC_EXTRAP = 0, BC_PERIODIC = 1, BC_WALL = 2, BC_INFLOW = 3 };
enum { TAU_RHO = 0, TAU_P = 1, TAU_HS1D = 2, TAU_CONST = 3 };
enum { PROJ_DISCRETE = 0, PROJ_PAPER = 1 };

struct Side {
    int kind;
    double T_wall, u_wall;
    double rho, u1, u2, T;
};

// Everything a kernel needs to know about the problem; passed by value.
struct Params {
    int nx, ny, nv1, nv2, nv;
    double x_lo, y_lo, v1_lo, v2_lo;
    double dx, dy, dv1, dv2;
    double eps, dt, nu;
    int tau_model;
    double tau_coef;
    int proj_mode;
    int wall_es_term;
    Side bc[4];   // 0 = x_lo, 1 = x_hi, 2 = y_lo, 3 = y_hi
};

__host__ __device__ inline bool is_open(int kind) { return kind == BC_WALL || kind == BC_INFLOW; }

// ---------------------------------------------------------------------------
// Per-cell record written by the preparation kernel from Q^n and read by the
// phase-space pass (2D).  FP64, REC doubles per cell.
enum {
    R_RHO = 0, R_U1, R_U2, R_T,
    R_RST,        // 1/sqrt(T)
    R_MPRE,       // rho / (2 pi T): Maxwellian prefactor
    R_I2T,        // 1 / (2T)
    R_TAU,
    R_A,          // eps / (eps + dt tau): weight of G** in the relaxation
    R_B,          // dt tau / (eps + dt tau): weight of G-hat
    R_P0,         // 10 entries: symmetric 4x4 matrix mapping sum_p phi_a F_p to the
                  // projection coefficients (dv1 dv2 Gram^{-1}, or dv1 dv2 / rho * I)
    R_GPRE = R_P0 + 10,   // rho / (2 pi sqrt(det calT))
    R_QA, R_QB, R_QC,     // exponent of the ES Gaussian: -(QA w1^2 + 2 QB w1 w2 + QC w2^2)
    R_S11, R_S12,         // sigma_11 (= -sigma_22), sigma_12 of (eqn5-97more)
    R_DTX, R_DTY,         // grad T of (eqn5-97)
    R_WALL,               // 1 for cells that use the wall form of G-hat
    R_ITAU,               // 1 / tau
    R_IEPS,               // 1 / eps
    R_IT,                 // 1 / T
    R_LG,                 // log(GPRE / MPRE) = log(T / sqrt(det calT))
    R_DA, R_DC,           // QA - 1/(2T), QC - 1/(2T): ES exponent minus Maxwellian exponent
    R_KM, R_KG,           // exp(-2 h^2 / 2T), exp(-2 QC h^2) with h = (64 / nv1) dv2 (lane-k node step
                          // in v2): second-difference factors of the Maxwellian and ES exponents
    R_PM,         // 10 entries: symmetric 4x4 matrix T^t P0 T mapping the raw moments
                  // sum (1, v1, v2, |v|^2) F straight to (c0, c1, c2, c3) with
                  // Pi F = (c0 + c1 v1 + c2 v2 + c3 |v|^2) M; T takes raw moments to moments
                  // against phi = (1, w1/sqrt T, w2/sqrt T, |w|^2/(2T) - 1), and its
                  // transpose takes phi coefficients back to the polynomial in v
    REC = 48
};
// wall cells: the four neighbour Maxwellians (x-, x+, y-, y+), each as
// (rho / (2 pi T), u1, u2, 1 / (2T))
enum { WREC = 16 };

// Lanes of a wavefront that the lane-k phase-space pass uses: L = 64 / nv1 lanes
// (integer division) share each v1 node, A = L nv1 lanes are active, and lane
// k + nv1 l0 (k < nv1, l0 < L) owns the nodes (k, l0 + L m), m < nv2 / L, i.e. the
// flat nodes lane + A m.  A layout exists when nv1 <= 64, L divides nv2 and A is 64
// (nv1 divides 64) or 48 (nv1 = 24 or 48), the two widths built; 0 otherwise.
__host__ __device__ inline int lk_lanes(int nv1, int nv2)
{
    if (nv1 < 1 || nv1 > 64) return 0;
    const int L = 64 / nv1, A = L * nv1;
    if ((A != 64 && A != 48) || nv2 < L || nv2 % L != 0) return 0;
    return A;
}

// Step in v2 between consecutive nodes of one lane in the lane-k phase-space
// pass (L dv2), or 0 where that layout does not apply
__host__ __device__ inline double lk_step(int nv1, int nv2, double dv2)
{
    if (lk_lanes(nv1, nv2) == 0) return 0.0;
    return (64 / nv1) * dv2;
}

// Range rule of the 2D solver: the Maxwellian and ES Gaussian exponents, and the
// exponent steps between lane-k nodes (h = (64 / nv1) dv2 apart in v2), stay
// within EXP_RANGE at every node of the velocity grid, so that each Gaussian can
// be followed along a lane's nodes from its first node without leaving the
// range of exp.  A state outside it (a gas too cold for the velocity grid) is
// reported as non-physical.  qa, qb, qc: the ES quadratic form; i2T = 1 / (2T).
constexpr double EXP_RANGE = 600.0;
__host__ __device__ inline bool exp_range_ok(double v1_lo, double dv1, int nv1, double v2_lo, double dv2, int nv2,
                                             double u1, double u2, double i2T, double qa, double qb, double qc)
{
    const double a0 = v1_lo + 0.5 * dv1 - u1, a1 = v1_lo + (nv1 - 0.5) * dv1 - u1;
    const double w0 = v2_lo + 0.5 * dv2 - u2, w1 = v2_lo + (nv2 - 0.5) * dv2 - u2;
    const double A = fmax(fabs(a0), fabs(a1)), W = fmax(fabs(w0), fabs(w1));
    const double h = lk_step(nv1, nv2, dv2);
    const double em = (A * A + W * W) * i2T;
    const double rm = (2.0 * W + h) * h * i2T;
    const double eg = qa * A * A + 2.0 * fabs(qb) * A * W + qc * W * W;
    const double rg = (2.0 * fabs(qb) * A + qc * (2.0 * W + h)) * h;
    return em <= EXP_RANGE && rm <= EXP_RANGE && eg <= EXP_RANGE && rg <= EXP_RANGE;
}

// index of the symmetric 4x4 entry (a, b) in the packed R_P0 block
__host__ __device__ constexpr int sym4(int a, int b)
{
    return a <= b ? (a == 0 ? b : a == 1 ? 3 + b : a == 2 ? 5 + b : 9)
                  : (b == 0 ? a : b == 1 ? 3 + a : b == 2 ? 5 + a : 9);
}

} // namespace mm
