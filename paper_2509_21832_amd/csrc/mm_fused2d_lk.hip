// mm_fused2d_lk.hip -- the fused phase-space pass specialised to velocity grids
// that map onto a wavefront by whole v1 rows: nv1 divides the wavefront width
// (nv1 in {2, 4, ..., 64}, all 64 lanes active), or nv1 is 24 or 48 (48 lanes
// active, the other 16 idle).
//
// Same step as mm_fused2d.hip (Sec. 5.3: x-transport, y-transport, G-hat of
// eqn5-97, relaxation eqn5-98, H of eqn5-99; wall-adjacent cells get G** only
// and are finished by k_wall_relax2d);
// what changes is the arithmetic layout.  With A = L nv1 active lanes (L = 64 / nv1,
// integer division) and node p = lane + A m, a lane owns one velocity
// k = lane mod nv1 and the nodes l = l0 + L m, so
//   - v1, the x-upwind weights and w1 = v1 - u1 are per-lane constants;
//   - every per-node polynomial (projection, the closed form of G-hat) is a
//     short Horner form in v2 whose coefficients a lane computes once per cell;
//   - the moment sums factor: a lane accumulates sum F, sum v2 F, sum v2^2 F
//     and multiplies by its own v1 powers once;
//   - the Maxwellian and the ES Gaussian have exponents quadratic in m, so
//     each follows an exact two-factor recurrence along a lane's nodes (in
//     FP64 for both compute types): no tables and no per-node exponential.
#include <type_traits>

#include "mm_fused_common.h"
#include "mm_launch.h"

namespace mm {

namespace {

using namespace fused;

// SYM: the v2 grid is symmetric about 0 with nv2 / 2 a multiple of 64 / nv1, so
// node m of every lane has v2 < 0 exactly when m < NPT / 2 and the y-upwind side
// is known when the kernel is compiled (checked on the host at launch)
// ACT: active lanes (64, or 48 with 16 idle lanes whose loads fall outside the
// buffer and read 0, whose stores are dropped, and whose sums are masked)
template <typename TS, typename TC, int NPT, bool CL, bool SYM, int ACT>
struct PassLK {
    // FP64: cell records are loaded rows ahead into VGPRs (one wavefront per SIMD
    // has the registers); FP32 keeps two wavefronts per SIMD and reads them in place
    using Rec = typename std::conditional<sizeof(TC) == 8, RecV, RecP>::type;
    const uint8_t *__restrict__ cls;   // closure form: 1 where the micro part is solved
    const TS *__restrict__ G;
    TS *__restrict__ Gn;
    double *__restrict__ H;
    const double *__restrict__ rec;
    const double *__restrict__ wrec;
    const Params *P;
    // Large instances (FP64 from 16 nodes per lane, FP32 from 48) park the local
    // part of G^{n+1} of the row being finished in this wavefront's LDS slice
    // between the two node loops instead of in registers.  For the FP32 instance
    // with 48 nodes this is what fits two wavefronts per SIMD (256 VGPRs instead of
    // 326): the pass went from 2.26 to 1.79-1.84 ms at 512^2 x 48^2
#ifndef MM_LK_STASH
#define MM_LK_STASH 1
#endif
    static constexpr bool STASH = MM_LK_STASH && ((sizeof(TC) == 8 && NPT >= 16) || NPT >= 48);
#ifndef MM_LK_WPROJ
#define MM_LK_WPROJ 1
#endif
#ifndef MM_LK_ESFOLD
#define MM_LK_ESFOLD 1
#endif
    TC *st;                 // this wavefront's slice: [NPT][64]
    int lane, i, k, l0, L;
    double act;             // 1 on an active lane, 0 on an idle one
    int row_bytes;          // bytes of one row of cells of g
    int off_c, off_u;       // byte offsets in its row of this lane's value of cell i and of its upwind cell
    double v1d, v2bd, hd;   // v1 of this lane; v2 of node m: v2b + m h
    double cxd;             // |v1| / dx
    int pe_src;             // 4 x the record field that holds this lane's entry of the composite map
    TC v1, cx, v2b, h, idy;

    // The node loops step v2 along the lane, w <- w + h from v2b: one add per
    // node (v2b + m h with the constant m would cost a register copy as well)

    // Moment sums along a lane's nodes run over the centred node index
    // t = m - (NPT - 1) / 2 (exact constants once the node loop is unrolled):
    // sum t^p F.  With the lane's centre velocity vc, v2 of node m is vc + t h, and the
    // sums of v2 powers follow once per row.  Centring keeps the expansion's terms
    // no larger than those of the direct sums.
    static constexpr double tn(int m) { return m - 0.5 * (NPT - 1); }
    __device__ __forceinline__ double vc() const { return v2bd + 0.5 * (NPT - 1) * hd; }
    // (sum F, sum t F, sum t^2 F) -> (sum F, sum v1 F, sum v2 F, sum |v|^2 F)
    __device__ __forceinline__ void raw4(const double *S, double (&s)[4]) const
    {
        const double c = vc();
        s[0] = S[0];
        s[1] = v1d * S[0];
        s[2] = c * S[0] + hd * S[1];
        s[3] = (v1d * v1d + c * c) * S[0] + (2.0 * c * hd) * S[1] + (hd * hd) * S[2];
    }

    // raw moments s (per lane) -> projection coefficients o (wave-uniform): the
    // wavefront sum and the record's composite map, applied across lanes
    // (wave_proj4).  Each lane takes its entry of the map from the record's lanes
    // by a permute (FP64: record held one field per lane) or by a load of its own
    // (FP32: record in memory).  MM_LK_WPROJ=0 builds the lane-by-lane product.
    __device__ __forceinline__ void sum_proj(double (&s)[4], const Rec &R, double (&o)[4]) const
    {
        if constexpr (std::is_same<Rec, RecV>::value && MM_LK_WPROJ) {
            wave_proj4(s, lane_read(R.v, pe_src), o);
        } else if constexpr (MM_LK_WPROJ == 1) {
            wave_proj4(s, R.p[pe_src >> 2], o);
        } else {
            wave_sum<4>(s, lane);
            proj_raw(R, s, o);
        }
    }

    // A Gaussian of the cell along this lane's nodes, e(m) = exp(quadratic in m),
    // follows the exact recurrence e(m+1) = e(m) r(m), r(m+1) = r(m) k, in FP64
    // for both compute types (the range rule of the 2D solver keeps e(0) and
    // r(0) inside the range of exp): no tables, no per-node exponential
    struct Gq {
        double e, r, k;
        __device__ __forceinline__ double next()
        {
            const double v = e;
            e *= r;
            r *= k;
            return v;
        }
    };
    // start values (e(0), r(0)) of a Gaussian's recurrence: the x-sweep of row j+1
    // makes the Maxwellian's, and the finish of that row one step later reuses them
    // (timed: faster by a few percent in FP64 and by 1.8% with g in FP32)
    struct GqS {
        double e, r;
    };
    GqS mq_cur{0.0, 0.0};   // the Maxwellian start values of the next row to finish
    // the Maxwellian of record R: mpre exp(-(w1^2 + w2(m)^2) / 2T)
    __device__ __forceinline__ Gq maxw_q(const Rec &R) const
    {
        const double i2T = R[R_I2T], a = v1d - R[R_U1], w = v2bd - R[R_U2];
        return Gq{R[R_MPRE] * exp(-(a * a + w * w) * i2T), exp(-(2.0 * w + hd) * hd * i2T), R[R_KM]};
    }
    // the ES Gaussian of record R: gpre exp(-(QA w1^2 + 2 QB w1 w2(m) + QC w2(m)^2))
    __device__ __forceinline__ Gq es_q(const Rec &R) const
    {
        const double qa = R[R_QA], qb = R[R_QB], qc = R[R_QC], a = v1d - R[R_U1], w = v2bd - R[R_U2];
        return Gq{R[R_GPRE] * exp(-((qa * a + 2.0 * qb * w) * a + qc * w * w)),
                  exp(-(2.0 * qb * a + qc * (2.0 * w + hd)) * hd), R[R_KG]};
    }

    // g of row r of cells (of G or Gn) as a buffer.  r is wave-uniform; stating it
    // keeps the resource in SGPRs also where the compiler merges call sites (a
    // resource it cannot prove uniform costs a waterfall loop per access)
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t row(const TS *base, int r) const
    {
        r = __builtin_amdgcn_readfirstlane(r);
        // the address and extent are stated wave-uniform as well (where the compiler
        // merges paths it can lose track of that)
        const uint64_t a = (uint64_t)(base + (size_t)r * P->nx * (ACT * NPT));
        const uint64_t au = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a) |
                            ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32)) << 32);
        return buf_rsrc((const TS *)au, __builtin_amdgcn_readfirstlane(row_bytes));
    }
    static constexpr int NB = ACT * (int)sizeof(TS);   // byte stride of node m

    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int off, TC (&out)[NPT]) const
    {
#pragma unroll
        for (int m = 0; m < NPT; ++m) out[m] = (TC)buf_load(rs, off, NB * m, (TS *)nullptr);
    }

    // x-transport of one cell: the upwind difference of this lane's velocity
    // needs only the upwind x-neighbour (i - 1 for v1 > 0, i + 1 otherwise), so
    // Z = |v1| / dx (g(i) - g(upwind)).  Beyond a non-periodic side the upwind
    // cell is the cell itself (the ghost takes its value: off_u = off_c), and
    // beyond an open side (wall, inflow) the ghost value is 0 instead (zero_nb).
    bool zero_nb;
    bool edge_col;   // wave-uniform: some lane of this column has zero_nb

    // g of cell i and of its upwind x-neighbour in row r, as an x-sweep reads them
    __device__ __forceinline__ void load_x(int r, TC (&gc)[NPT], TC (&gu)[NPT]) const
    {
        const auto rs = row(G, r);
        load(rs, off_c, gc);
        load(rs, off_u, gu);
    }

    // x-sweep from the loaded values: G*(i, r) = g - dt (I - Pi)[Z] into out, with
    // Z = cx d and d = g(i) - g(upwind).  The first node loop leaves g - dt Z in out
    // and sums d; after the wavefront sum and the projection the second adds
    // dt Pi[Z] = (dt q-polynomial) M.  Neither g nor d stays live across the sums.
    // R: the record of cell (i, r)
    __device__ __forceinline__ GqS xsweep_v(const TC (&gc)[NPT], TC (&gu)[NPT], TC (&out)[NPT], const Rec &R)
    {
        if (edge_col) {
#pragma unroll
            for (int m = 0; m < NPT; ++m) gu[m] = zero_nb ? (TC)0 : gu[m];
        }
        const TC dcx = (TC)P->dt * cx;
        double S[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const TC d = gc[m] - gu[m];
            out[m] = gc[m] - dcx * d;
            const double dd = (double)d;
            S[0] += dd;
            S[1] += tn(m) * dd;
            S[2] += (tn(m) * tn(m)) * dd;
        }
        // sums of Z = cx d
        S[0] *= cxd;
        S[1] *= cxd;
        S[2] *= cxd;
        double s[4];
        raw4(S, s);
        double o[4];
        sum_proj(s, R, o);
        const double dtd = P->dt;
        const TC c2 = (TC)(dtd * o[2]), c3 = (TC)(dtd * o[3]), K = (TC)(dtd * (o[0] + (o[1] + o[3] * v1d) * v1d));
        const Gq m0 = maxw_q(R);
        Gq mq = m0;
        TC w = v2b;
#pragma unroll
        for (int m = 0; m < NPT; ++m, w += h) {
            const TC pm = (c3 * w + c2) * w + K;
            out[m] = pm * (TC)mq.next() + out[m];
        }
        if constexpr (ACT < 64) {
            if (act == 0.0) {
#pragma unroll
                for (int m = 0; m < NPT; ++m) out[m] = (TC)0;
            }
        }
        return GqS{m0.e, m0.r};
    }

    // x-sweep of row r: G*(i, r) into out; R: the record of cell (i, r)
    __device__ __forceinline__ GqS xsweep(int r, TC (&out)[NPT], const Rec &R)
    {
        TC gc[NPT], gu[NPT];
        load_x(r, gc, gu);
        return xsweep_v(gc, gu, out, R);
    }

    // y-transport of node m: v2 (G(j) - G(j -/+ 1)) / dy upwind, written as
    // |v2| / dy (G(j) - G(upwind)) (the same value); wy = v2 / dy of the node,
    // stepped along the lane (wy <- wy + h / dy) by the node loops
    __device__ __forceinline__ TC zy(int m, TC wy, const TC (&lo)[NPT], const TC (&ce)[NPT], const TC (&hi)[NPT]) const
    {
        if constexpr (SYM) {
            const TC up = m < NPT / 2 ? hi[m] : lo[m];
            const TC aw = m < NPT / 2 ? -wy : wy;
            TC d = ce[m] - up;
            // FP64: pin the difference where it is used; left free, the compiler
            // forms the row's differences early and needs more than 256 VGPRs
            if constexpr (sizeof(TC) == 8) asm volatile("" : "+v"(d));
            return aw * d;
        } else {
            return fabs(wy) * (ce[m] - (wy < (TC)0 ? hi[m] : lo[m]));
        }
    }

    // y-sweep of a wall-adjacent cell: G** only.  The wall form of G-hat, the
    // relaxation and H of these cells are done by k_wall_relax2d afterwards.
    __device__ __forceinline__ void wall_row(int jr, const TC (&lo)[NPT], const TC (&ce)[NPT], const TC (&hi)[NPT],
                                             const Rec &R, GqS ms)
    {
        TC Zy[NPT];
        double S[3] = {0.0, 0.0, 0.0};
        TC wy = v2b * idy;
        const TC hy = h * idy;
#pragma unroll
        for (int m = 0; m < NPT; ++m, wy += hy) {
            Zy[m] = zy(m, wy, lo, ce, hi);
            const double z = (double)Zy[m];
            S[0] += z;
            S[1] += tn(m) * z;
            S[2] += (tn(m) * tn(m)) * z;
        }
        double s[4];
        raw4(S, s);
        double o[4];
        sum_proj(s, R, o);
        const TC c2 = (TC)o[2], c3 = (TC)o[3], Kz = (TC)(o[0] + (o[1] + o[3] * v1d) * v1d), dt = (TC)P->dt;
        const auto ws = row(Gn, jr);
        Gq mq{ms.e, ms.r, R[R_KM]};
        TC w = v2b;
#pragma unroll
        for (int m = 0; m < NPT; ++m, w += h) {
            const TC pz = (c3 * w + c2) * w + Kz;
            buf_store((TS)(ce[m] + dt * (pz * (TC)mq.next() - Zy[m])), ws, off_c, NB * m);
        }
    }

    // closed form of G-hat (eqn5-97) at this lane's w1 = a as a cubic in w2, times -1/tau
    __device__ __forceinline__ void ghat_cubic(const Rec &R, double a, TC (&C)[4]) const
    {
        const double i2T = R[R_I2T], iT = R[R_IT], itau = R[R_ITAU];
        const double s11 = R[R_S11], s12 = R[R_S12], dTx = R[R_DTX], dTy = R[R_DTY];
        const double q = a * a * i2T - 2.0;
        C[0] = (TC)(-itau * (s11 * a * a * i2T + iT * q * a * dTx));
        C[1] = (TC)(-itau * (2.0 * s12 * a * i2T + iT * q * dTy));
        C[2] = (TC)(-itau * (-s11 * i2T + iT * i2T * a * dTx));
        C[3] = (TC)(-itau * (iT * i2T * dTy));
    }

    // y-sweep, G-hat (eqn5-97), relaxation and H for interior row j with window
    // (lo, ce, hi).  The ES term (calG - M) / eps is formed in FP64 from the two
    // Gaussians, then converted to the compute type.  The relaxation
    //   G^{n+1} = ra (ce + dt (pz M - Zy)) + rb (G-hat - pb M)
    // has pz M = Pi[Zy] and pb M = Pi[G-hat] (G-hat is not projected in the
    // paper's form: pb = 0).  Pi is linear, so with d = ra dt Zy - rb' G-hat
    // (rb' = rb, or 0 in the paper's form)
    //   G^{n+1} = [ra ce - d + (rb - rb') G-hat] + Pi[d]:
    // the first node loop forms the bracket and the moments of d, and after one
    // wavefront sum Pi[d] = (q0 + q1 v1 + q2 v2 + q3 |v|^2) M.
    __device__ __forceinline__ void finish_row(size_t c, int jr, const TC (&lo)[NPT], const TC (&ce)[NPT],
                                               const TC (&hi)[NPT], const Rec &R, GqS ms)
    {
        const bool discrete = P->proj_mode == PROJ_DISCRETE;
        const double u2d = R[R_U2];
        const double a = v1d - R[R_U1];             // w1 of this lane
        TC C[4];
        ghat_cubic(R, a, C);
        const Gq mq0{ms.e, ms.r, R[R_KM]};
        Gq gq = es_q(R);
        const double iepsd = R[R_IEPS], rbd = R[R_B];
        const TC u2 = (TC)u2d;
        const TC ra = (TC)R[R_A], radt = ra * (TC)P->dt;
        const TC rbp = discrete ? (TC)rbd : (TC)0, rbq = discrete ? (TC)0 : (TC)rbd;
        TC part[STASH ? 1 : NPT];
        double S[3] = {0.0, 0.0, 0.0};
        // FP64: the ES term's -M / eps joins the cubic's constant, so the node value
        // is M (cubic - 1/eps) + calG / eps (rounding of the same order as forming
        // calG - M first); FP32 forms calG - M in FP64 before the conversion
        constexpr bool ESFOLD = sizeof(TC) == 8 && MM_LK_ESFOLD;
        if constexpr (ESFOLD) C[0] -= (TC)iepsd;
        {
            Gq mq = mq0;
            TC w2 = v2b - u2, wy = v2b * idy;
            const TC hy = h * idy;
#pragma unroll
            for (int m = 0; m < NPT; ++m, w2 += h, wy += hy) {
                const TC zv = zy(m, wy, lo, ce, hi);
                const double Md = mq.next();
                const TC M = (TC)Md;
                const TC cub = ((C[3] * w2 + C[2]) * w2 + C[1]) * w2 + C[0];
                TC bv;
                if constexpr (ESFOLD) bv = M * cub + (TC)iepsd * (TC)gq.next();
                else bv = M * cub + (TC)((gq.next() - Md) * iepsd);
                const TC d = radt * zv - rbp * bv;
                const TC pv = ra * ce[m] + (rbq * bv - d);
                if constexpr (STASH) st[m * 64 + lane] = pv;
                else part[m] = pv;
                const double dd = (double)d;
                S[0] += dd;
                S[1] += tn(m) * dd;
                S[2] += (tn(m) * tn(m)) * dd;
            }
        }
        if constexpr (ACT < 64) {
            S[0] *= act;
            S[1] *= act;
            S[2] *= act;
        }
        double s[4];
        raw4(S, s);
        double o[4];
        sum_proj(s, R, o);
        const TC q3 = (TC)o[3], q2 = (TC)o[2], q0 = (TC)(o[0] + (o[1] + o[3] * v1d) * v1d);
        const auto ws = row(Gn, jr);
        // recompute the node values below rather than hold all NPT of them from the first loop
        refresh();
        double T[4] = {0.0, 0.0, 0.0, 0.0};
        Gq mq = mq0;
        TC w = v2b;
#pragma unroll
        for (int m = 0; m < NPT; ++m, w += h) {
            const TC M = (TC)mq.next();
            const TC pv = STASH ? st[m * 64 + lane] : part[STASH ? 0 : m];
            const TS gn = (TS)(((q3 * w + q2) * w + q0) * M + pv);
            buf_store(gn, ws, off_c, NB * m);
            const double g = (double)gn;
            T[0] += g;
            T[1] += tn(m) * g;
            T[2] += (tn(m) * tn(m)) * g;
            T[3] += (tn(m) * tn(m) * tn(m)) * g;
        }
        if constexpr (ACT < 64) {
#pragma unroll
            for (int q = 0; q < 4; ++q) T[q] *= act;
        }
        // sum g w2^p with w2 = v2 - u2 = e + t h (e: the lane's centre velocity minus u2)
        const double e = vc() - u2d, e2 = e * e, h2 = hd * hd;
        const double g1 = e * T[0] + hd * T[1];
        const double g2 = e2 * T[0] + (2.0 * e * hd) * T[1] + h2 * T[2];
        const double g3 = (e2 * e) * T[0] + (3.0 * e2 * hd) * T[1] + (3.0 * e * h2) * T[2] + (h2 * hd) * T[3];
        double hs[4] = {a * a * a * T[0], a * a * g1, a * g2, g3};
        wave_sum<4>(hs, lane);
        if (lane == 0) {
            const double f = P->eps * P->dv1 * P->dv2;
            for (int qq = 0; qq < 4; ++qq) H[c * 4 + qq] = f * hs[qq];
        }
    }

    __device__ __forceinline__ void ghost(int kind, const TC (&own)[NPT], TC (&dst)[NPT]) const
    {
        const bool open = is_open(kind);
#pragma unroll
        for (int m = 0; m < NPT; ++m) dst[m] = open ? (TC)0 : own[m];
    }

    // one row: G* of row j+1 into win[HI], then finish row j
    // (the segment ends at row j1 - 1, so its last x-sweep is row j1)
    // Per-node constants depend only on the lane, so the compiler would hoist
    // all NPT of them out of the row loop and keep them in registers.  Passing
    // the lane's base values through an empty asm once per row makes them
    // row-variant: the node constants are recomputed (one FMA each) instead.
    __device__ __forceinline__ void refresh()
    {
        asm volatile("" : "+v"(v2bd), "+v"(l0), "+v"(hd));
        v2b = (TC)v2bd;
        h = (TC)hd;
    }

    // closure form: is the micro part of cell (i, r) solved?  Rows beyond a
    // periodic side wrap; beyond any other side there are no cells.
    __device__ __forceinline__ bool micro_load(int r) const
    {
        if (r < 0 || r >= P->ny) {
            if (P->bc[2].kind != BC_PERIODIC) return false;
            r = r < 0 ? r + P->ny : r - P->ny;
        }
        return cls[(size_t)r * P->nx + i] != 0;
    }
    // the same from the classes of rows cbase .. cbase + 63, read once per segment
    uint64_t cmask = 0;
    int cbase = 0;
    __device__ __forceinline__ bool micro_row(int r) const { return (cmask >> (r - cbase)) & 1; }

    // (closure form: G* of row j+1 is made only if one of rows j, j+1, j+2 is
    // solved, and row j is finished only if it is solved)
    // row of the x-sweep for window row r (beyond a periodic side: wrapped;
    // beyond any other side: -1, a ghost row)
    __device__ __forceinline__ int xrow(int r) const
    {
        if (r >= 0 && r < P->ny) return r;
        if (P->bc[2].kind != BC_PERIODIC) return -1;
        return r < 0 ? r + P->ny : r - P->ny;
    }

    static constexpr bool RING = std::is_same<Rec, RecV>::value;

    // FP64: load the record of cell (i, xrow(r)) ahead of its use into a ring slot
    __device__ __forceinline__ void fetch_rec(int r, Rec &dst) const
    {
        if constexpr (RING) {
            const int x = xrow(r);
            if (x >= 0) dst = load_rec(rec, (size_t)x * P->nx + i, lane);
        }
    }

    // the record of cell (i, x) for its use: the ring slot (FP64) or the record in memory
    __device__ __forceinline__ Rec rec_at(int x, const Rec &slot) const
    {
        if constexpr (RING) return slot;
        else return Rec{rec + ((size_t)x * P->nx + i) * REC};
    }

    template <int LO, int CE, int HI>
    __device__ __forceinline__ void step(int j, int j1, TC (&win)[3][NPT], Rec (&rv)[3])
    {
        refresh();
        __builtin_amdgcn_sched_barrier(0);
        // records ride with the window: rv[CE] is row j, rv[HI] row j + 1; the
        // record of row j + 2 (next step's x-sweep) is loaded now into rv[LO]
        if (j + 2 <= j1) fetch_rec(j + 2, rv[LO]);
        bool solve = true;
        if constexpr (CL) {
            solve = micro_row(j);
            if (!solve && !micro_row(j + 1) && !micro_row(j + 2)) return;
        }
        GqS nx{0.0, 0.0};
        if (j + 1 < P->ny) {
            nx = xsweep(j + 1, win[HI], rec_at(j + 1, rv[HI]));
        }
        else if (P->bc[3].kind == BC_PERIODIC) nx = xsweep(0, win[HI], rec_at(0, rv[HI]));
        else ghost(P->bc[3].kind, win[CE], win[HI]);
        // row j finishes with the start values its own x-sweep made one step ago
        // (a row that was not swept is not finished either)
        const GqS ms = mq_cur;
        mq_cur = nx;
        __builtin_amdgcn_sched_barrier(0);
        if (CL && !solve) return;
        refresh();
        const size_t c = (size_t)j * P->nx + i;
        const Rec R = rec_at(j, rv[CE]);
        if (R[R_WALL] != 0.0) wall_row(j, win[LO], win[CE], win[HI], R, ms);
        else finish_row(c, j, win[LO], win[CE], win[HI], R, ms);
        __builtin_amdgcn_sched_barrier(0);
    }
};

// Occupancy: the FP64 instance with 16 nodes per lane (128 B of G per lane)
// runs one wavefront per SIMD (measured faster than two); every other instance,
// the FP32 one with 48 nodes per lane included (its window half in LDS), runs
// two wavefronts per SIMD.
#ifndef MM_LK_OCC64
#define MM_LK_OCC64 1
#endif
template <typename TC, int NPT>
struct LKTraits {
    static constexpr bool big = sizeof(TC) * NPT >= 128;   // the same rule picks the launch geometry
    static constexpr int occupancy = big && !(sizeof(TC) == 4 && NPT >= 48) ? MM_LK_OCC64 : 2;
};

template <typename TS, typename TC, int NPT, bool CL, bool SYM, int ACT>
__global__ __launch_bounds__(64 * WPG, (LKTraits<TC, NPT>::occupancy)) void k_fused2d_lk(const TS *__restrict__ G, TS *__restrict__ Gn,
                                                            double *__restrict__ H, const double *__restrict__ rec,
                                                            const double *__restrict__ wrec,
                                                            const Params *__restrict__ Pd, Geom geo,
                                                            const uint8_t *__restrict__ cls)
{
    const Params &P = *Pd;
    const int t = tile_of(blockIdx.x, geo.ntiles);
    if (t >= geo.ntiles) return;
    const int cg = t % geo.ncg, sg = t / geo.ncg;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: cell indices live in SGPRs
    using Pass = PassLK<TS, TC, NPT, CL, SYM, ACT>;
    Pass ps;
    __shared__ TC s_st[Pass::STASH ? WPG * NPT * 64 : 1];
    ps.st = s_st + (Pass::STASH ? wv * NPT * 64 : 0);
    ps.cls = cls;
    ps.G = G; ps.Gn = Gn; ps.H = H; ps.rec = rec; ps.wrec = wrec; ps.P = Pd;
    ps.lane = threadIdx.x & 63;
    ps.i = cg * WPG + wv;
    if (ps.i >= P.nx) return;
    ps.k = ps.lane % P.nv1;
    ps.L = 64 / P.nv1;
    ps.act = ps.lane < ACT ? 1.0 : 0.0;
    ps.l0 = ps.lane / P.nv1;
    ps.v1d = P.v1_lo + (ps.k + 0.5) * P.dv1;
    ps.v2bd = P.v2_lo + (ps.l0 + 0.5) * P.dv2;
    ps.hd = ps.L * P.dv2;
    ps.v1 = (TC)ps.v1d;
    ps.cxd = fabs(ps.v1d) / P.dx;
    {
        // lane 16 r + c (c < 4) takes entry (c, r) of the record's composite map; the
        // other lanes take field R_PM + 10, which the preparation kernel sets to 0
        static_assert(R_PM + 10 < REC, "a zero field follows the composite map");
        const int r = ps.lane >> 4, c = ps.lane & 15;
        ps.pe_src = 4 * (c < 4 ? R_PM + sym4(c, r) : R_PM + 10);
    }
    ps.cx = (TC)ps.cxd;
    {
        const bool pos = ps.v1d > 0.0;
        const int side = pos ? 0 : 1;
        int iu = pos ? ps.i - 1 : ps.i + 1;
        bool ghost = false;
        if (iu < 0 || iu >= P.nx) {
            if (P.bc[side].kind == BC_PERIODIC) iu = iu < 0 ? P.nx - 1 : 0;
            else {
                ghost = true;
                iu = ps.i;
            }
        }
        ps.row_bytes = P.nx * ACT * NPT * (int)sizeof(TS);
        ps.off_c = (ps.i * ACT * NPT + ps.lane) * (int)sizeof(TS);
        ps.off_u = (iu * ACT * NPT + ps.lane) * (int)sizeof(TS);
        // an idle lane addresses past the row: its loads read 0, its stores are dropped
        if (ps.lane >= ACT) ps.off_c = ps.off_u = ps.row_bytes;
        ps.zero_nb = ghost && is_open(P.bc[side].kind);
        ps.edge_col = __ballot(ps.zero_nb) != 0;
    }
    ps.v2b = (TC)ps.v2bd;
    ps.h = (TC)ps.hd;
    ps.idy = (TC)(1.0 / P.dy);
    const int j0 = sg * geo.seg, j1 = min(P.ny, j0 + geo.seg);

    if constexpr (CL) {
        // classes of this segment's rows of the column, one per lane, in one ballot
        // (segments are at most 61 rows); rows of other segments count as not
        // solved here, since this wavefront finishes only its own rows
        const int r = j0 - 1 + ps.lane;
        const bool m = r >= j0 && r < j1 && ps.micro_load(r);
        ps.cmask = __ballot(m);
        ps.cbase = j0 - 1;
        if (ps.cmask == 0) return;
    }
    TC win[3][NPT];
    // records of the window rows j0 - 1, j0, j0 + 1 (slots 0, 1, 2)
    typename Pass::Rec rv[3] = {};
    ps.fetch_rec(j0 - 1, rv[0]);
    ps.fetch_rec(j0, rv[1]);
    ps.fetch_rec(j0 + 1, rv[2]);
    // closure form: the prologue rows are needed only for solved rows of the segment
    if (!CL || ps.micro_row(j0 - 1) || ps.micro_row(j0) || ps.micro_row(j0 + 1))
        ps.mq_cur = ps.xsweep(j0, win[1], ps.rec_at(j0, rv[1]));
    if (!CL || ps.micro_row(j0)) {
        if (j0 > 0) ps.xsweep(j0 - 1, win[0], ps.rec_at(j0 - 1, rv[0]));
        else if (P.bc[2].kind == BC_PERIODIC) ps.xsweep(P.ny - 1, win[0], ps.rec_at(P.ny - 1, rv[0]));
        else ps.ghost(P.bc[2].kind, win[1], win[0]);
    }
    // full rounds of three rows rotate the window back to its start; the tail
    // (one or two rows) runs after the loop so the window is never merged
    int j = j0;
    for (; j + 3 <= j1; j += 3) {
        ps.template step<0, 1, 2>(j, j1, win, rv);
        ps.template step<1, 2, 0>(j + 1, j1, win, rv);
        ps.template step<2, 0, 1>(j + 2, j1, win, rv);
    }
    if (j < j1) ps.template step<0, 1, 2>(j, j1, win, rv);
    if (j + 1 < j1) ps.template step<1, 2, 0>(j + 1, j1, win, rv);
}

template <typename TS, typename TC, bool CL, bool SYM>
bool launch_lk_t(int npt, int act, const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                 const Params *Pd, const Geom &geo, const uint8_t *cls, hipStream_t st)
{
    const dim3 grid(((geo.ntiles + 7) / 8) * 8), block(64 * WPG);
#define MM_LAUNCH(N, ACT)                                                                                   \
    hipLaunchKernelGGL((k_fused2d_lk<TS, TC, N, CL, SYM, ACT>), grid, block, 0, st, (const TS *)G,         \
                       (TS *)Gn, H, rec, wrec, Pd, geo, cls)
    if (act == 64) {
        switch (npt) {
        case 1: MM_LAUNCH(1, 64); return true;
        case 2: MM_LAUNCH(2, 64); return true;
        case 4: MM_LAUNCH(4, 64); return true;
        case 8: MM_LAUNCH(8, 64); return true;
        case 16: MM_LAUNCH(16, 64); return true;
        default: return false;
        }
    }
    if constexpr (!CL) {
        if (npt == 12) {
            MM_LAUNCH(12, 48);
            return true;
        }
        if (npt == 24) {
            MM_LAUNCH(24, 48);
            return true;
        }
        {
            if (npt == 48) {
                MM_LAUNCH(48, 48);
                return true;
            }
        }
    }
    return false;
#undef MM_LAUNCH
}

// Wall-adjacent cells in the lane-k layout (one wavefront per ring cell, the
// node ownership of k_fused2d_lk).  The pass left G** of these cells in Gn; here
// follow the wall form of G-hat (Sec. 6.3), -(1/tau)(I - Pi)[M_up] + (calG - M)/eps,
// with M_up the upwind difference of the four neighbour (or ghost) Maxwellians,
// then the relaxation (eqn5-98) and H (eqn5-99).  Every Gaussian follows the
// exact recurrence of the pass along the lane's nodes; the sums are wavefront
// sums, so there are no block barriers.
struct GqW {
    double e, r, k;
    __device__ __forceinline__ double next()
    {
        const double v = e;
        e *= r;
        r *= k;
        return v;
    }
};

template <typename TS, int NPT, int ACT>
__global__ __launch_bounds__(256) void k_wall_lk(TS *__restrict__ Gn, double *__restrict__ H,
                                                  const double *__restrict__ rec, const double *__restrict__ wrec,
                                                  Params P, int nring)
{
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rr = blockIdx.x * 4 + wv;
    if (rr >= nring) return;
    int i, j;
    ring_cell(P, rr, i, j);
    const size_t c = (size_t)j * P.nx + i;
    const double *R = rec + c * REC;
    if (R[R_WALL] == 0.0) return;
    const int lane = threadIdx.x & 63;
    const int k = lane % P.nv1, L = 64 / P.nv1, l0 = lane / P.nv1;
    const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2b = P.v2_lo + (l0 + 0.5) * P.dv2, h = L * P.dv2;
    const double u1 = R[R_U1], u2 = R[R_U2], ieps = R[R_IEPS], itau = R[R_ITAU];
    const bool es_on = P.wall_es_term != 0, discrete = P.proj_mode == PROJ_DISCRETE;
    const double idx = 1.0 / P.dx, idy = 1.0 / P.dy;
    auto maxw = [&](double pre, double cu1, double cu2, double ci2T, double kap) {
        const double a = v1 - cu1, w = v2b - cu2;
        return GqW{pre * exp(-(a * a + w * w) * ci2T), exp(-(2.0 * w + h) * h * ci2T), kap};
    };
    const GqW m0 = maxw(R[R_MPRE], u1, u2, R[R_I2T], R[R_KM]);
    const double *nb = wrec + c * WREC;   // x-, x+, y-, y+: (rho / (2 pi T), u1, u2, 1 / (2T))
    GqW mn[4];
#pragma unroll
    for (int d = 0; d < 4; ++d)
        mn[d] = maxw(nb[4 * d], nb[4 * d + 1], nb[4 * d + 2], nb[4 * d + 3], exp(-2.0 * h * h * nb[4 * d + 3]));
    GqW gq;
    {
        const double qa = R[R_QA], qb = R[R_QB], qc = R[R_QC], a = v1 - u1, w = v2b - u2;
        gq = GqW{R[R_GPRE] * exp(-((qa * a + 2.0 * qb * w) * a + qc * w * w)),
                 exp(-(2.0 * qb * a + qc * (2.0 * w + h)) * h), R[R_KG]};
    }
    const int bytes = P.nv * (int)sizeof(TS);
    const auto rs = buf_rsrc(Gn + c * (size_t)P.nv, bytes);
    // an idle lane (lane >= ACT) addresses past the cell: it reads 0 and writes nothing
    const int off = lane < ACT ? lane * (int)sizeof(TS) : bytes;
    const double act = lane < ACT ? 1.0 : 0.0;
    constexpr int NB = ACT * (int)sizeof(TS);
    // the upwind Maxwellian difference and the ES term of node m are held between the
    // two node loops, or (long lanes) recomputed in the second from the recurrences
    constexpr bool HOLD = NPT <= 16;
    TS g[NPT];
    double mup[HOLD ? NPT : 1], es[HOLD ? NPT : 1];
#pragma unroll
    for (int m = 0; m < NPT; ++m) g[m] = buf_load(rs, off, NB * m, (TS *)nullptr);
    const double ax = fmin(v1, 0.0) * idx, bx = fmax(v1, 0.0) * idx;
    auto node = [&](int m, GqW &mq, GqW (&mv)[4], GqW &gv, double &mu, double &e) {
        const double w = v2b + m * h;
        const double M = mq.next(), M0 = mv[0].next(), M1 = mv[1].next(), M2 = mv[2].next(), M3 = mv[3].next();
        mu = (ax * (M1 - M) + bx * (M - M0)) + (fmin(w, 0.0) * (M3 - M) + fmax(w, 0.0) * (M - M2)) * idy;
        e = es_on ? (gv.next() - M) * ieps : 0.0;
        return M;
    };
    double acc[6] = {0, 0, 0, 0, 0, 0};
    {
        GqW mq = m0, mv[4] = {mn[0], mn[1], mn[2], mn[3]}, gv = gq;
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const double w = v2b + m * h;
            double mu, e;
            node(m, mq, mv, gv, mu, e);
            if constexpr (HOLD) {
                mup[m] = mu;
                es[m] = e;
            }
            const double uz = w * mu, ub = w * e;
            acc[0] += mu;
            acc[1] += uz;
            acc[2] += w * uz;
            acc[3] += e;
            acc[4] += ub;
            acc[5] += w * ub;
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] *= act;
    // G-hat = -itau (mup - Pi[mup]) + (es - Pi[es]) (es unprojected in the paper's
    // form) = -itau mup + es + Pi[itau mup - es]: one projection of combined moments
    const double v1s = v1 * v1, eb = discrete ? 1.0 : 0.0;
    double s[4] = {itau * acc[0] - eb * acc[3], v1 * (itau * acc[0] - eb * acc[3]), itau * acc[1] - eb * acc[4],
                   v1s * (itau * acc[0] - eb * acc[3]) + (itau * acc[2] - eb * acc[5])};
    wave_sum<4>(s, lane);
    double o[4];
    proj_raw(RecP{R}, s, o);
    const double K = o[0] + o[1] * v1 + o[3] * v1s;
    const double ra = R[R_A], rb = R[R_B];
    const double a = v1 - u1;
    double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
    GqW mq = m0, mv[4] = {mn[0], mn[1], mn[2], mn[3]}, gv = gq;
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
        const double w = v2b + m * h;
        double M, mu, e;
        if constexpr (HOLD) {
            M = mq.next();
            mu = mup[m];
            e = es[m];
        } else {
            M = node(m, mq, mv, gv, mu, e);
        }
        const double gh = -itau * mu + e + ((o[3] * w + o[2]) * w + K) * M;
        const TS gn = (TS)(ra * (double)g[m] + rb * gh);
        buf_store(gn, rs, off, NB * m);
        const double gvl = (double)gn, w2 = w - u2;
        const double ug = gvl * w2, ug2 = ug * w2;
        h0 += gvl;
        h1 += ug;
        h2 += ug2;
        h3 += ug2 * w2;
    }
    double hs[4] = {act * a * a * a * h0, act * a * a * h1, act * a * h2, act * h3};
    wave_sum<4>(hs, lane);
    if (lane == 0) {
        const double f = P.eps * P.dv1 * P.dv2;
        for (int q = 0; q < 4; ++q) H[c * 4 + q] = f * hs[q];
    }
}

} // namespace

// nodes per lane of the lane-k layout of P (0: no layout): A = 64 lanes take
// 1, 2, 4, 8 or 16 nodes each; A = 48 lanes take 12 or 24 (both storage
// precisions) or 48 (g in FP32 only)
static int lk_npt(const Params &P, int precision)
{
    const int A = lk_lanes(P.nv1, P.nv2);
    if (A == 0 || P.nv2 > MAXV) return 0;
    // a row of cells of g is addressed with 32-bit byte offsets
    if ((long long)P.nx * P.nv * 8 >= (1LL << 31)) return 0;
    const int npt = P.nv / A;
    if (A == 64) return (npt == 1 || npt == 2 || npt == 4 || npt == 8 || npt == 16) ? npt : 0;
    return (npt == 12 || npt == 24 || npt == 48) ? npt : 0;
}

bool lk_supported(const Params &P) { return lk_lanes(P.nv1, P.nv2) == 64 && lk_npt(P, 0) != 0; }
bool lk_supported(const Params &P, int precision) { return lk_npt(P, precision) != 0; }

bool launch_wall_lk2d(void *Gn, int g_bytes, double *H, const double *rec, const double *wrec, const Params &P,
                      hipStream_t st)
{
    const int A = lk_lanes(P.nv1, P.nv2), npt = lk_npt(P, g_bytes == 8 ? 0 : 1);
    if (npt == 0) return false;
    const int nring = 2 * P.nx + 2 * (P.ny - 2);
    const dim3 grid((nring + 3) / 4), block(256);
#define MM_LAUNCH(N, ACT)                                                                                      \
    do {                                                                                                       \
        if (g_bytes == 8)                                                                                      \
            hipLaunchKernelGGL((k_wall_lk<double, N, ACT>), grid, block, 0, st, (double *)Gn, H, rec, wrec, P,  \
                               nring);                                                                         \
        else                                                                                                   \
            hipLaunchKernelGGL((k_wall_lk<float, N, ACT>), grid, block, 0, st, (float *)Gn, H, rec, wrec, P,    \
                               nring);                                                                         \
    } while (0)
    if (A == 64) {
        switch (npt) {
        case 1: MM_LAUNCH(1, 64); return true;
        case 2: MM_LAUNCH(2, 64); return true;
        case 4: MM_LAUNCH(4, 64); return true;
        case 8: MM_LAUNCH(8, 64); return true;
        case 16: MM_LAUNCH(16, 64); return true;
        default: return false;
        }
    }
    if (npt == 12) {
        MM_LAUNCH(12, 48);
        return true;
    }
    if (npt == 24) {
        MM_LAUNCH(24, 48);
        return true;
    }
    if (g_bytes == 4)
        hipLaunchKernelGGL((k_wall_lk<float, 48, 48>), grid, block, 0, st, (float *)Gn, H, rec, wrec, P, nring);
    else
        hipLaunchKernelGGL((k_wall_lk<double, 48, 48>), grid, block, 0, st, (double *)Gn, H, rec, wrec, P, nring);
    return true;
#undef MM_LAUNCH
}

// The v2 grid is symmetric about 0 and each lane has as many nodes below 0 as
// above (nv2 / 2 a multiple of L = 64 / nv1): node m of every lane has v2 < 0
// exactly when m < NPT / 2.  The two middle nodes are checked with a margin of a
// quarter node spacing, far beyond rounding.
static bool v2_symmetric_lk(const Params &P)
{
    const int L = 64 / P.nv1;
    if (P.nv2 % (2 * L) != 0) return false;
    const double below = P.v2_lo + (P.nv2 / 2 - 0.5) * P.dv2, above = P.v2_lo + (P.nv2 / 2 + 0.5) * P.dv2;
    return below < -0.25 * P.dv2 && above > 0.25 * P.dv2 && fabs(below + above) < 1e-9 * P.dv2;
}

bool launch_micro_lk2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                       const Params &P, const Params *Pd, int precision, const uint8_t *cls, hipStream_t st)
{
    const int act = lk_lanes(P.nv1, P.nv2), npt = lk_npt(P, precision);
    if (npt == 0) return false;
    // the instances with 128 bytes of g per lane and more run one wavefront per SIMD,
    // except the FP32 one with 48 nodes per lane (see LKTraits)
    const bool one_wave =
        (precision == 0 ? 8 : 4) * npt >= 128 && MM_LK_OCC64 == 1 && !(precision != 0 && npt >= 48);
    // g in FP32 with 16 nodes per lane: one and a half rounds of workgroups (row
    // segments of 22 rows at 256^2 x 32^2) measured 5% faster than two (163.5 against
    // 172.4 us, bitwise the same result); the FP64 instances and the 48-node FP32 one
    // are fastest at two rounds (FP64 at 256^2 x 32^2: 223 us, 233-291 us at segments
    // of 28-40 rows; FP32 at 512^2 x 48^2: 1.80 against 1.98 ms at one and a half)
    const Geom geo = geometry(P, one_wave ? 1 : 2, precision != 0 && npt == 16 ? 6 : 8);
    if (cls) {   // closure form: g in FP32 only, 64 active lanes
        if (act != 64) return false;
        // the solved cells cluster along the walls: short row segments spread a
        // fully solved column over many wavefronts
        Geom gc = geo;
        gc.seg = P.ny < 4 ? P.ny : 4;        // at most 61 (one class bit per lane)
        gc.nseg = (P.ny + gc.seg - 1) / gc.seg;
        gc.ntiles = gc.ncg * gc.nseg;
        return precision != 0 &&
               launch_lk_t<float, float, true, false>(npt, act, G, Gn, H, rec, wrec, Pd, gc, cls, st);
    }
    if (v2_symmetric_lk(P))
        return precision == 0
                   ? launch_lk_t<double, double, false, true>(npt, act, G, Gn, H, rec, wrec, Pd, geo, nullptr, st)
                   : launch_lk_t<float, float, false, true>(npt, act, G, Gn, H, rec, wrec, Pd, geo, nullptr, st);
    return precision == 0
               ? launch_lk_t<double, double, false, false>(npt, act, G, Gn, H, rec, wrec, Pd, geo, nullptr, st)
               : launch_lk_t<float, float, false, false>(npt, act, G, Gn, H, rec, wrec, Pd, geo, nullptr, st);
}

} // namespace mm
