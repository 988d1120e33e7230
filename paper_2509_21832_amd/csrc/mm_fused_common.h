// mm_fused_common.h -- helpers shared by the fused phase-space kernels:
// wavefront reductions, per-cell coefficients, the projection polynomial and
// the launch geometry (internal).
#pragma once
#include "mm_device.h"

namespace mm {
namespace fused {

constexpr int WPG = 4;        // wavefronts per workgroup (one column each)
constexpr int MAXV = 64;      // largest nv1, nv2 of the fused pass

__device__ __forceinline__ double bcast(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// One halving step of the wavefront sum below: lanes with bit `o` set keep
// the upper H partial sums, the others the lower H, and each adds its
// partner's copy of the half it keeps.
template <int H>
__device__ __forceinline__ void fold(double *a, int o, int lane)
{
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double keep = up ? a[k + H] : a[k];
        const double send = up ? a[k] : a[k + H];
        a[k] = keep + __shfl_xor(send, o, 64);
    }
}

// Sum N doubles (N a power of two, <= 16) over the wavefront.  A halving step
// exchanges n/2 values instead of n; after log2(N) of them lane L holds partial
// sum number L >> (6 - log2 N), the remaining xor steps finish the sums, and
// the totals are read back as wave-uniform values.
template <int N>
__device__ __forceinline__ void wave_sum(double (&v)[N], int lane)
{
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "power of two <= 16");
    double a[N];
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] = v[k];
    if constexpr (N >= 2) fold<N / 2>(a, 32, lane);
    if constexpr (N >= 4) fold<N / 4>(a, 16, lane);
    if constexpr (N >= 8) fold<N / 8>(a, 8, lane);
    if constexpr (N >= 16) fold<N / 16>(a, 4, lane);
#pragma unroll
    for (int o = 32 / N; o >= 1; o >>= 1) a[0] += __shfl_xor(a[0], o, 64);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = bcast(a[0], q * (64 / N));
}

__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double t_expm1(double x) { return expm1(x); }

// Per-cell coefficients (wave-uniform), converted to the compute type
template <typename TC>
struct Cell {
    TC u1, u2, i2T, iT, itau, ieps, s11, s12, dTx, dTy;
    TC dA, dB, dC, lg;         // ES exponent difference: delta = lg - (dA w1^2 + 2 dB w1 w2 + dC w2^2)
    double P0[10];
    double u1d, u2d, rsTd, i2Td, ra, rb;
};

template <typename TC>
__device__ __forceinline__ void load_cell(const double *R, Cell<TC> &c)
{
    c.u1d = R[R_U1];
    c.u2d = R[R_U2];
    c.rsTd = R[R_RST];
    c.i2Td = R[R_I2T];
    c.u1 = (TC)c.u1d;
    c.u2 = (TC)c.u2d;
    c.i2T = (TC)c.i2Td;
    c.iT = (TC)R[R_IT];
    c.itau = (TC)R[R_ITAU];
    c.ieps = (TC)R[R_IEPS];
    c.s11 = (TC)R[R_S11];
    c.s12 = (TC)R[R_S12];
    c.dTx = (TC)R[R_DTX];
    c.dTy = (TC)R[R_DTY];
    c.dA = (TC)R[R_DA];
    c.dB = (TC)R[R_QB];
    c.dC = (TC)R[R_DC];
    c.lg = (TC)R[R_LG];
#pragma unroll
    for (int q = 0; q < 10; ++q) c.P0[q] = R[R_P0 + q];
    c.ra = R[R_A];
    c.rb = R[R_B];
}

// Projection coefficients from raw moments s = sum (1, v1, v2, |v|^2) F:
// returns (c0, c1, c2, c3) with Pi F = (c0 + c1 v1 + c2 v2 + c3 |v|^2) M.
template <typename TC>
__device__ __forceinline__ void proj_poly(const Cell<TC> &c, const double *s, TC out[4])
{
    const double u1 = c.u1d, u2 = c.u2d, rsT = c.rsTd, i2T = c.i2Td;
    // moments against the basis phi = (1, w1/sqrt T, w2/sqrt T, |w|^2/(2T) - 1)
    const double sw1 = s[1] - u1 * s[0], sw2 = s[2] - u2 * s[0];
    const double sww = s[3] - 2.0 * u1 * s[1] - 2.0 * u2 * s[2] + (u1 * u1 + u2 * u2) * s[0];
    const double b[4] = {s[0], rsT * sw1, rsT * sw2, i2T * sww - s[0]};
    double A[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v += c.P0[sym4(a, q)] * b[q];
        A[a] = v;
    }
    // sum_a A_a phi_a as a polynomial in v
    const double c3 = A[3] * i2T;
    out[3] = (TC)c3;
    out[1] = (TC)(A[1] * rsT - 2.0 * c3 * u1);
    out[2] = (TC)(A[2] * rsT - 2.0 * c3 * u2);
    out[0] = (TC)(A[0] - A[1] * rsT * u1 - A[2] * rsT * u2 + c3 * (u1 * u1 + u2 * u2) - A[3]);
}

// Geometry of the launch: columns are grouped WPG to a workgroup; rows are cut
// into segments of `seg` rows.  Workgroup b works on tile t(b), where tiles
// that share halo columns get consecutive ids on the same XCD (dispatch puts
// workgroup b on XCD b mod 8).
struct Geom {
    int ncg, nseg, seg, ntiles;
};

__device__ __forceinline__ int tile_of(int b, int ntiles)
{
    const int per = (ntiles + 7) / 8;
    return (b % 8) * per + b / 8;   // >= ntiles for padding workgroups
}

// Workgroups per launch: about two rounds of (CUs x resident workgroups per CU),
// with row segments of at least 16 rows.
inline Geom geometry(const Params &P, int occupancy)
{
    Geom g;
    g.ncg = (P.nx + WPG - 1) / WPG;
    const int want = 2 * 256 * occupancy;
    const int nseg = (want + g.ncg - 1) / g.ncg;
    int seg = (P.ny + nseg - 1) / nseg;
    if (seg < 16) seg = 16;
    if (seg > P.ny) seg = P.ny;
    g.seg = seg;
    g.nseg = (P.ny + seg - 1) / seg;
    g.ntiles = g.ncg * g.nseg;
    return g;
}

} // namespace fused

// the lane-k specialisation of the fused pass (mm_fused2d_lk.hip)
bool lk_supported(const Params &P);
bool launch_micro_lk2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                       const Params &P, const Params *Pd, int precision, const fused::Geom &geo, hipStream_t st);

} // namespace mm
