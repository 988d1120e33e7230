// mm_source.hip -- the source terms of the paper's manufactured-solution
// convergence studies, evaluated on the GPU (2D: Sec. 6.2; the 1D source of
// Sec. 3.4 lives in the 1D kernels).
//
// 2D invented solution (Sec. 6.2):
//   f(t, x, v) = A(v) B(t, x),  A = exp(-|v - e|^2) + 2 exp(-|v + e|^2),  e = (1, 1),
//   B = 2 - sin 2pi(t - x) cos 2pi(t - y),
// and its residual S = f_t + v . grad f - (tau / eps)(calG[f] - f).  Since
// B_t = -(B_x + B_y), f_t + v . grad f = A ((v1 - 1) B_x + (v2 - 1) B_y).  calG[f] is
// the ES Gaussian of f's own moments, and tau that of f's state: S is a function
// of the invented solution alone.
//
// The micro step takes (1 / tau_ij^n)(I - Pi)[S](t^n, x_ij, v) into G-hat.  Since
// G^{n+1} = ra G** + rb G-hat, this kernel adds (rb / tau)(I - Pi)[S] to G^{n+1}
// after the phase-space pass and the matching eps dv sum w^3 (...) to H^{n+1}.
// The macro step takes dt int psi S dv between the y-sweep and the second
// collision half step; this kernel writes those moments (closed form) per cell.
#include "mm_device.h"
#include "mm_fused_common.h"
#include "mm_launch.h"

namespace mm {

namespace {

// int v1^a v2^b A dv: A is pi N((1,1), I/2) + 2 pi N((-1,-1), I/2), and the 1D
// moments of N(m, 1/2) are 1, m, m^2 + 1/2, m^3 + 3m/2
__device__ __forceinline__ double half_var_moment(int n, double m)
{
    switch (n) {
    case 0: return 1.0;
    case 1: return m;
    case 2: return m * m + 0.5;
    default: return m * m * m + 1.5 * m;
    }
}
__device__ __forceinline__ double momA(int a, int b)
{
    return MM_PI * (half_var_moment(a, 1.0) * half_var_moment(b, 1.0) +
                    2.0 * half_var_moment(a, -1.0) * half_var_moment(b, -1.0));
}

struct Mms2State {
    double B, Bx, By;
    double rho, u1, u2, p, T;
    double P11, P12, P22;
    double tau;
    double gpre, qa, qb, qc;     // ES Gaussian: gpre exp(-(qa w1^2 + 2 qb w1 w2 + qc w2^2))
};

// the exact state of f at (t, x, y): moments of A times B
__device__ Mms2State mms2_state(const Params &P, double t, double x, double y)
{
    Mms2State s;
    const double a = 2.0 * MM_PI * (t - x), b = 2.0 * MM_PI * (t - y);
    const double sa = sin(a), ca = cos(a), sb = sin(b), cb = cos(b);
    s.B = 2.0 - sa * cb;
    s.Bx = 2.0 * MM_PI * ca * cb;        // d/dx of -sin a cos b, da/dx = -2 pi
    s.By = -2.0 * MM_PI * sa * sb;       // d/dy, db/dy = -2 pi
    s.rho = momA(0, 0) * s.B;
    s.u1 = momA(1, 0) / momA(0, 0);
    s.u2 = momA(0, 1) / momA(0, 0);
    s.P11 = (momA(2, 0) - momA(0, 0) * s.u1 * s.u1) * s.B;
    s.P12 = (momA(1, 1) - momA(0, 0) * s.u1 * s.u2) * s.B;
    s.P22 = (momA(0, 2) - momA(0, 0) * s.u2 * s.u2) * s.B;
    s.p = 0.5 * (s.P11 + s.P22);
    s.T = s.p / s.rho;
    s.tau = tau_of(P, s.rho, s.p, s.T);
    // ES tensor calT = (1 - nu) T I + nu P / rho (eq2-19) and its inverse / 2
    const double S11 = (1.0 - P.nu) * s.T + P.nu * s.P11 / s.rho;
    const double S12 = P.nu * s.P12 / s.rho;
    const double S22 = (1.0 - P.nu) * s.T + P.nu * s.P22 / s.rho;
    const double det = S11 * S22 - S12 * S12;
    s.gpre = s.rho / (2.0 * MM_PI * sqrt(det));
    s.qa = S22 / (2.0 * det);
    s.qb = -S12 / (2.0 * det);
    s.qc = S11 / (2.0 * det);
    return s;
}

__device__ __forceinline__ double mms2_S(const Params &P, const Mms2State &s, double v1, double v2)
{
    const double A = exp(-((v1 - 1.0) * (v1 - 1.0) + (v2 - 1.0) * (v2 - 1.0))) +
                     2.0 * exp(-((v1 + 1.0) * (v1 + 1.0) + (v2 + 1.0) * (v2 + 1.0)));
    const double w1 = v1 - s.u1, w2 = v2 - s.u2;
    const double G = s.gpre * exp(-((s.qa * w1 + 2.0 * s.qb * w2) * w1 + s.qc * w2 * w2));
    return A * ((v1 - 1.0) * s.Bx + (v2 - 1.0) * s.By) - s.tau / P.eps * (G - A * s.B);
}

// one workgroup per cell; t: time of the step's old level t^n
template <typename TG>
__global__ __launch_bounds__(256) void k_source2d(TG *__restrict__ Gn, double *__restrict__ H,
                                                   const double *__restrict__ rec, double *__restrict__ msrc,
                                                   Params P, double t)
{
    __shared__ double lds[4 * 4];
    const int c = blockIdx.x, i = c % P.nx, j = c / P.nx;
    const double x = P.x_lo + (i + 0.5) * P.dx, y = P.y_lo + (j + 0.5) * P.dy;
    const Mms2State s = mms2_state(P, t, x, y);
    const double *R = rec + (size_t)c * REC;
    // raw moments sum (1, v1, v2, |v|^2) S for the projection
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < P.nv; q += 256) {
        const double v1 = P.v1_lo + (q % P.nv1 + 0.5) * P.dv1, v2 = P.v2_lo + (q / P.nv1 + 0.5) * P.dv2;
        const double S = mms2_S(P, s, v1, v2);
        m[0] += S;
        m[1] += v1 * S;
        m[2] += v2 * S;
        m[3] += (v1 * v1 + v2 * v2) * S;
    }
    block_sum<4, 4>(m, lds);
    double o[4];
    fused::proj_raw(fused::RecP{R}, m, o);
    const double u1 = R[R_U1], u2 = R[R_U2], mpre = R[R_MPRE], i2T = R[R_I2T];
    const double f = R[R_B] * R[R_ITAU];
    double hs[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < P.nv; q += 256) {
        const double v1 = P.v1_lo + (q % P.nv1 + 0.5) * P.dv1, v2 = P.v2_lo + (q / P.nv1 + 0.5) * P.dv2;
        const double w1 = v1 - u1, w2 = v2 - u2;
        const double M = mpre * exp(-(w1 * w1 + w2 * w2) * i2T);
        const double add = f * (mms2_S(P, s, v1, v2) - (o[0] + o[1] * v1 + o[2] * v2 + o[3] * (v1 * v1 + v2 * v2)) * M);
        const size_t at = (size_t)c * P.nv + q;
        const TG gn = (TG)((double)Gn[at] + add);
        Gn[at] = gn;
        hs[0] += w1 * w1 * w1 * add;
        hs[1] += w1 * w1 * w2 * add;
        hs[2] += w1 * w2 * w2 * add;
        hs[3] += w2 * w2 * w2 * add;
    }
    block_sum<4, 4>(hs, lds);
    if (threadIdx.x == 0) {
        const double e = P.eps * P.dv1 * P.dv2;
        for (int a = 0; a < 4; ++a) H[(size_t)c * 4 + a] += e * hs[a];
        // int (1, v1, v2, v1^2, v1 v2, v2^2) S dv: the transport part from the moments
        // of A; of the collision part only the second moments remain,
        // int v v (calG - f) = rho calT - P = (1 - nu)(p I - P)
        const int ex[6][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2}};
        const double coll[6] = {0.0, 0.0, 0.0, (1.0 - P.nu) * (s.p - s.P11), -(1.0 - P.nu) * s.P12,
                                (1.0 - P.nu) * (s.p - s.P22)};
        for (int r = 0; r < 6; ++r) {
            const int a = ex[r][0], b = ex[r][1];
            const double m0 = momA(a, b);
            msrc[(size_t)c * 6 + r] = s.Bx * (momA(a + 1, b) - m0) + s.By * (momA(a, b + 1) - m0) -
                                      s.tau / P.eps * coll[r];
        }
    }
}

} // namespace

void launch_source2d(void *Gn, int g_bytes, double *H, const double *rec, double *msrc, const Params &P, double t,
                     hipStream_t st)
{
    const int n = P.nx * P.ny;
    if (g_bytes == 8)
        hipLaunchKernelGGL(k_source2d<double>, dim3(n), dim3(256), 0, st, (double *)Gn, H, rec, msrc, P, t);
    else
        hipLaunchKernelGGL(k_source2d<float>, dim3(n), dim3(256), 0, st, (float *)Gn, H, rec, msrc, P, t);
}

} // namespace mm
