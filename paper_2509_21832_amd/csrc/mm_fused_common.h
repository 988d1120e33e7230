// mm_fused_common.h -- helpers shared by the fused phase-space kernels:
// wavefront reductions, per-cell coefficients, the projection polynomial and
// the launch geometry (internal).
#pragma once
#include "mm_device.h"

namespace mm {
namespace fused {

constexpr int WPG = 4;        // wavefronts per workgroup (one column each)
constexpr int MAXV = 64;      // largest nv1, nv2 of the fused pass


// ---------------------------------------------------------------------------
// Wavefront sums built from gfx950 lane permutations that stay in the VALU
// (no LDS round trip): v_permlane32_swap / v_permlane16_swap exchange whole
// rows between lane halves / row pairs, DPP quad_perm and row mirrors pair
// lanes inside a row of 16.

__device__ __forceinline__ double hilo(unsigned hi, unsigned lo)
{
    return __hiloint2double((int)hi, (int)lo);
}

// DPP move of both halves of a double (ctrl: a DPP control code).  Every row
// and bank is written and the patterns used here read valid lanes only, so no
// old value is kept (one DPP move per half, no copy).
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Fold across lane bit 5 (32) or 4 (16): on return a lane holds, in `lo`, the
// sum of its own and its partner's copy of the half it keeps: lanes with the
// bit clear keep `lo`, lanes with the bit set keep `hi`.
template <int BIT>
__device__ __forceinline__ double fold_swap(double lo, double hi)
{
    static_assert(BIT == 4 || BIT == 5, "permlane swaps cover lane bits 4 and 5");
    unsigned a0 = (unsigned)__double2loint(lo), a1 = (unsigned)__double2hiint(lo);
    unsigned b0 = (unsigned)__double2loint(hi), b1 = (unsigned)__double2hiint(hi);
    if constexpr (BIT == 5) {
        const auto r0 = __builtin_amdgcn_permlane32_swap(a0, b0, false, false);
        const auto r1 = __builtin_amdgcn_permlane32_swap(a1, b1, false, false);
        return hilo(r1[0], r0[0]) + hilo(r1[1], r0[1]);
    } else {
        const auto r0 = __builtin_amdgcn_permlane16_swap(a0, b0, false, false);
        const auto r1 = __builtin_amdgcn_permlane16_swap(a1, b1, false, false);
        return hilo(r1[0], r0[0]) + hilo(r1[1], r0[1]);
    }
}

// all-reduce inside each row of 16 lanes: pairs (xor 1), (xor 2) by quad_perm,
// then the half-row and row mirrors
__device__ __forceinline__ double row_sum(double v)
{
    v += dpp<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);    // row_half_mirror
    v += dpp<0x140>(v);    // row_mirror
    return v;
}

__device__ __forceinline__ double bcast(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum N doubles (N = 1, 2, 4 or 8) over the wavefront; every lane receives the
// totals as wave-uniform values.  Two fold steps halve the number of values
// per lane across lane bits 5 and 4 (value q ends in the row q / (N/4)), the
// row sums finish them.  The combination order is fixed (bitwise reproducible).
template <int N>
__device__ __forceinline__ void wave_sum(double (&v)[N], int lane)
{
    (void)lane;
    static_assert(N == 1 || N == 2 || N == 4 || N == 8, "N in {1, 2, 4, 8}");
    if constexpr (N == 1) {
        double x = v[0];
        x = fold_swap<5>(x, x);
        x = fold_swap<4>(x, x);
        v[0] = bcast(row_sum(x), 0);
    } else if constexpr (N == 2) {
        double x = fold_swap<5>(v[0], v[1]);        // rows 0,1: value 0; rows 2,3: value 1
        x = fold_swap<4>(x, x);
        x = row_sum(x);
        v[0] = bcast(x, 0);
        v[1] = bcast(x, 32);
    } else {
        constexpr int H = N / 2, Q = N / 4;
        double a[H], b[Q];
#pragma unroll
        for (int k = 0; k < H; ++k) a[k] = fold_swap<5>(v[k], v[k + H]);
#pragma unroll
        for (int k = 0; k < Q; ++k) b[k] = row_sum(fold_swap<4>(a[k], a[k + Q]));
        // value q = r * Q + t sits in slot t of row r
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < Q; ++t) v[r * Q + t] = bcast(b[t], 16 * r);
    }
}

// Wavefront sum of four per-lane values s followed by the symmetric 4x4 map
// o = Pm s, with the map applied across lanes instead of by every lane: after the
// folds of wave_sum<4>, row r of the wavefront holds the total s_r in all its
// lanes; lane 16 r + c multiplies it by its entry pe = Pm[c][r] (c < 4; pe = 0 on
// the other lanes), a fold over the four rows sums the products, and lane c then
// holds o_c, read out as a scalar.  (A lane-by-lane product would read the ten
// entries and the four totals as scalars and issue 16 FMAs with two scalar
// operands each.)  The combination order is fixed.
__device__ __forceinline__ void wave_proj4(const double (&s)[4], double pe, double (&o)[4])
{
    const double a0 = fold_swap<5>(s[0], s[2]);
    const double a1 = fold_swap<5>(s[1], s[3]);
    double x = row_sum(fold_swap<4>(a0, a1)) * pe;
    x = fold_swap<5>(x, x);
    x = fold_swap<4>(x, x);
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = bcast(x, c);
}

// value of lane src_byte / 4 of v, in every lane (cross-lane permute through the
// LDS unit; no LDS memory)
__device__ __forceinline__ double lane_read(double v, int src_byte)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src_byte, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src_byte, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double t_expm1(double x) { return expm1(x); }

// Raw buffer access: a wave-uniform base and extent (one row of cells) in
// SGPRs, the lane's byte offset in one VGPR and the node's byte offset as an
// SGPR or immediate.  Accesses beyond the extent read 0 and write nothing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, 0x00020000);
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, double *)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, float *)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// Stores are non-temporal (cache policy bit NT): g of the next time level is
// not read again by the kernel that writes it
constexpr int STORE_NT = 2;
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, STORE_NT);
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, STORE_NT);
}

// Per-cell coefficients (wave-uniform), converted to the compute type
template <typename TC>
struct Cell {
    TC u1, u2, i2T, iT, itau, ieps, s11, s12, dTx, dTy;
    TC dA, dB, dC, lg;         // ES exponent difference: delta = lg - (dA w1^2 + 2 dB w1 w2 + dC w2^2)
    double P0[10];
    double u1d, u2d, rsTd, i2Td, ra, rb;
};

// A per-cell record held in a wavefront's VGPRs, one field per lane (lane q
// holds field q < REC); a field is read as a wave-uniform value (v_readlane),
// so a record loaded rows ahead costs no scalar-load round trip when used
struct RecV {
    double v;
    __device__ __forceinline__ double operator[](int q) const { return bcast(v, q); }
};

// the same interface over the record in memory (scalar loads at each use)
struct RecP {
    const double *p;
    __device__ __forceinline__ double operator[](int q) const { return p[q]; }
};

// one coalesced load of the record of `cell`
__device__ __forceinline__ RecV load_rec(const double *rec, size_t cell, int lane)
{
    RecV r;
    r.v = lane < REC ? rec[cell * REC + lane] : 0.0;
    return r;
}

// R: a pointer to the record or a RecV
template <typename TC, typename RT>
__device__ __forceinline__ void load_cell(const RT &R, Cell<TC> &c)
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

// The same coefficients from the raw moments s = sum (1, v1, v2, |v|^2) F with
// the record's composite map (R_PM): one symmetric 4x4 product.
template <typename RT>
__device__ __forceinline__ void proj_raw(const RT &R, const double *s, double out[4])
{
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v += R[R_PM + sym4(a, q)] * s[q];
        out[a] = v;
    }
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

// Workgroups per launch: about `quarters` / 4 rounds of (CUs x resident
// workgroups per CU) (two rounds by default), with row segments of at least 16 rows.
inline Geom geometry(const Params &P, int occupancy, int quarters = 8)
{
    Geom g;
    g.ncg = (P.nx + WPG - 1) / WPG;
    const int want = quarters * 64 * occupancy;
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
// the lane-k pass takes this grid at this precision (0 FP64, 1 g in FP32)
bool lk_supported(const Params &P, int precision);
// cls: nullptr, or (closure form, g in FP32) the per-cell flags of solved cells
bool launch_micro_lk2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                       const Params &P, const Params *Pd, int precision, const uint8_t *cls, hipStream_t st);

} // namespace mm
