// mm_fused2d.hip -- the fused 2D phase-space pass: x-transport (G^n -> G*),
// y-transport (G* -> G**), G-hat, backward-Euler relaxation and the heat-flux
// tensor in one read of G^n and one write of G^{n+1}.
//
// Paper: Rossmanith & Sar, arXiv:2509.21832, Sec. 5.3 (eqs. zmicrox ..
// update-micro-2D-ydir, eqn5-97, eqn5-97more, eqn5-98), eqn5-99, and the wall
// form of G-hat of Sec. 6.3.
//
// Mapping on gfx950:
//   - one 64-wide wavefront owns one spatial column i and marches up a segment
//     of rows j; a lane owns NPT velocity nodes p = lane + 64 m of every cell;
//   - the y-sweep of row j needs G* of rows j-1, j, j+1, so the wavefront keeps
//     a three-row window of G* in registers and computes G* of row j+1 (the
//     x-sweep, which needs the x-neighbour cells of the same row) just before
//     it finishes row j;
//   - every velocity moment is a wavefront reduction (transposed butterfly of
//     cross-lane shuffles, totals read back as scalars), so the waves of a
//     workgroup never wait for each other;
//   - the Maxwellian of a cell is separable, M = [rho/(2 pi T) e1(k)] e2(l): each
//     wavefront keeps per-cell tables of e1, e2 in its own LDS slice;
//   - the ES term (G - M)/eps is evaluated as M expm1(delta)/eps, with delta
//     the (small) difference of the two exponents, so no cancellation occurs;
//   - wall-adjacent cells get G** only; k_wall_relax2d finishes them with the
//     wall form of G-hat (Sec. 6.3), the relaxation and H.
// G may be stored in FP64 (TS = double, arithmetic in FP64) or FP32
// (TS = float, per-node arithmetic in FP32); velocity sums are always FP64.
#include <cstdlib>

#include "mm_fused_common.h"
#include "mm_launch.h"

namespace mm {

namespace {

using namespace fused;

template <typename TS, typename TC, int NPT>
struct Pass {
    const TS *__restrict__ G;
    TS *__restrict__ Gn;
    double *__restrict__ H;
    const double *__restrict__ rec;
    const double *__restrict__ wrec;
    const Params *P;
    const double2 *sv;    // per-node (v1, v2) in LDS
    const int2 *skl;      // per-node (k, l) in LDS
    double *tab;          // this wavefront's Maxwellian tables: 3 slots x 2 x MAXV
    int lane, i;

    // the Maxwellian of node p = lane + 64 m; 0 on the padding slots p >= nv of the
    // last node of a lane, so that they add nothing to any sum or to H
    __device__ __forceinline__ TC maxw_tab(int slot, int m) const
    {
        const int p = lane + 64 * m;
        const int2 kl = skl[p];
        const double *t = tab + slot * 2 * MAXV;
        return p < P->nv ? (TC)(t[kl.x] * t[MAXV + kl.y]) : (TC)0;
    }

    __device__ __forceinline__ void build_tables(int slot, const double *R) const
    {
        const double u1 = R[R_U1], u2 = R[R_U2], i2T = R[R_I2T], mpre = R[R_MPRE];
        double *t = tab + slot * 2 * MAXV;
        if (lane < P->nv1) {
            const double w = P->v1_lo + (lane + 0.5) * P->dv1 - u1;
            t[lane] = mpre * exp(-w * w * i2T);
        }
        if (lane < P->nv2) {
            const double w = P->v2_lo + (lane + 0.5) * P->dv2 - u2;
            t[MAXV + lane] = exp(-w * w * i2T);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    __device__ __forceinline__ void load(size_t cell, TC (&out)[NPT]) const
    {
        const TS *g = G + cell * (size_t)P->nv;
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const int p = lane + 64 * m;
            out[m] = p < P->nv ? (TC)g[p] : (TC)0;
        }
    }

    // x-sweep of row r: G*(i, r) into out; tables of cell (i, r) go to `slot`
    __device__ __forceinline__ void xsweep(int r, int slot, TC (&out)[NPT]) const
    {
        const size_t c = (size_t)r * P->nx + i;
        const double *R = rec + c * REC;
        build_tables(slot, R);
        TC gc[NPT], Z[NPT];
        {
            TC gm[NPT], gp[NPT];
            load(c, gc);
            // x neighbours with the boundary ghosts of Sec. 5.3.1 / 5.3.2 / 6.3
            if (i > 0) load(c - 1, gm);
            else if (P->bc[0].kind == BC_PERIODIC) load(c + P->nx - 1, gm);
            else {
                const bool open = is_open(P->bc[0].kind);
#pragma unroll
                for (int m = 0; m < NPT; ++m) gm[m] = open ? (TC)0 : gc[m];
            }
            if (i < P->nx - 1) load(c + 1, gp);
            else if (P->bc[1].kind == BC_PERIODIC) load(c - (P->nx - 1), gp);
            else {
                const bool open = is_open(P->bc[1].kind);
#pragma unroll
                for (int m = 0; m < NPT; ++m) gp[m] = open ? (TC)0 : gc[m];
            }
            const TC idx = (TC)(1.0 / P->dx);
#pragma unroll
            for (int m = 0; m < NPT; ++m) {
                const TC v1 = (TC)sv[lane + 64 * m].x;
                Z[m] = (fmin(v1, (TC)0) * (gp[m] - gc[m]) + fmax(v1, (TC)0) * (gc[m] - gm[m])) * idx;
            }
        }
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const double2 v = sv[lane + 64 * m];
            const double z = (double)Z[m];
            s[0] += z;
            s[1] += v.x * z;
            s[2] += v.y * z;
            s[3] += (v.x * v.x + v.y * v.y) * z;
        }
        wave_sum<4>(s, lane);
        Cell<TC> cl;
        load_cell(R, cl);
        TC cp[4];
        proj_poly(cl, s, cp);
        const TC dt = (TC)P->dt;
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const double2 v = sv[lane + 64 * m];
            const TC v1 = (TC)v.x, v2 = (TC)v.y;
            const TC poly = cp[0] + cp[1] * v1 + cp[2] * v2 + cp[3] * (v1 * v1 + v2 * v2);
            const TC M = maxw_tab(slot, m);
            out[m] = gc[m] + dt * (poly * M - Z[m]);
        }
    }

    __device__ __forceinline__ TC zy(int m, const TC (&lo)[NPT], const TC (&ce)[NPT], const TC (&hi)[NPT],
                                     TC idy) const
    {
        const TC v2 = (TC)sv[lane + 64 * m].y;
        return (fmin(v2, (TC)0) * (hi[m] - ce[m]) + fmax(v2, (TC)0) * (ce[m] - lo[m])) * idy;
    }

    // y-sweep of a wall-adjacent cell: G** only (the wall G-hat, relaxation and
    // H of these cells are done by k_wall_relax2d afterwards)
    __device__ __forceinline__ void wall_row(size_t c, int slot, const TC (&lo)[NPT], const TC (&ce)[NPT],
                                             const TC (&hi)[NPT]) const
    {
        const double *R = rec + c * REC;
        Cell<TC> cl;
        load_cell(R, cl);
        const TC idy = (TC)(1.0 / P->dy);
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const double2 v = sv[lane + 64 * m];
            const double z = (double)zy(m, lo, ce, hi, idy);
            s[0] += z; s[1] += v.x * z; s[2] += v.y * z; s[3] += (v.x * v.x + v.y * v.y) * z;
        }
        wave_sum<4>(s, lane);
        TC cz[4];
        proj_poly(cl, s, cz);
        const TC dt = (TC)P->dt;
        TS *gout = Gn + c * (size_t)P->nv;
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const int p = lane + 64 * m;
            const double2 v = sv[p];
            const TC v1 = (TC)v.x, v2 = (TC)v.y;
            const TC pz = cz[0] + cz[1] * v1 + cz[2] * v2 + cz[3] * (v1 * v1 + v2 * v2);
            const TC gss = ce[m] + dt * (pz * maxw_tab(slot, m) - zy(m, lo, ce, hi, idy));
            if (p < P->nv) gout[p] = (TS)gss;
        }
    }

    // y-sweep, G-hat (eqn5-97), relaxation and H for interior row j with window (lo, ce, hi)
    __device__ __forceinline__ void finish_row(size_t c, int slot, const TC (&lo)[NPT], const TC (&ce)[NPT],
                                               const TC (&hi)[NPT]) const
    {
        const double *R = rec + c * REC;
        Cell<TC> cl;
        load_cell(R, cl);
        const bool discrete = P->proj_mode == PROJ_DISCRETE;
        const TC idy = (TC)(1.0 / P->dy);
        TC base[NPT];
        double s[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] = 0.0;
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const double2 v = sv[lane + 64 * m];
            const TC v1 = (TC)v.x, v2 = (TC)v.y;
            const TC M = maxw_tab(slot, m);
            const TC w1 = v1 - cl.u1, w2 = v2 - cl.u2;
            const TC w11 = w1 * w1, w22 = w2 * w2, w12 = w1 * w2;
            const TC delta = cl.lg - (cl.dA * w11 + (TC)2 * cl.dB * w12 + cl.dC * w22);
            const TC es = M * t_expm1(delta) * cl.ieps;
            const TC Bs = (cl.s11 * (w11 - w22) + (TC)2 * cl.s12 * w12) * cl.i2T;
            const TC CgT = ((w11 + w22) * cl.i2T - (TC)2) * cl.iT * (w1 * cl.dTx + w2 * cl.dTy);
            base[m] = -cl.itau * (Bs + CgT) * M + es;
            const double vsq = v.x * v.x + v.y * v.y;
            const double z = (double)zy(m, lo, ce, hi, idy), b = (double)base[m];
            s[0] += z; s[1] += v.x * z; s[2] += v.y * z; s[3] += vsq * z;
            s[4] += b; s[5] += v.x * b; s[6] += v.y * b; s[7] += vsq * b;
        }
        wave_sum<8>(s, lane);
        TC cz[4], cb[4] = {(TC)0, (TC)0, (TC)0, (TC)0};
        proj_poly(cl, s, cz);
        if (discrete) proj_poly(cl, s + 4, cb);
        const TC dt = (TC)P->dt, ra = (TC)cl.ra, rb = (TC)cl.rb;
        TS *gout = Gn + c * (size_t)P->nv;
        double h[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const int p = lane + 64 * m;
            const double2 v = sv[p];
            const TC v1 = (TC)v.x, v2 = (TC)v.y, vsq = v1 * v1 + v2 * v2;
            const TC M = maxw_tab(slot, m);
            const TC pz = cz[0] + cz[1] * v1 + cz[2] * v2 + cz[3] * vsq;
            const TC pb = cb[0] + cb[1] * v1 + cb[2] * v2 + cb[3] * vsq;
            const TC gss = ce[m] + dt * (pz * M - zy(m, lo, ce, hi, idy));
            const TC gh = base[m] - pb * M;
            const TS gn = (TS)(ra * gss + rb * gh);
            if (p < P->nv) gout[p] = gn;
            const double g = (double)gn, w1 = v.x - cl.u1d, w2 = v.y - cl.u2d;
            const double g11 = g * w1 * w1, g22 = g * w2 * w2;
            h[0] += g11 * w1;
            h[1] += g11 * w2;
            h[2] += g22 * w1;
            h[3] += g22 * w2;
        }
        wave_sum<4>(h, lane);
        if (lane == 0) {
            const double f = P->eps * P->dv1 * P->dv2;
            for (int a = 0; a < 4; ++a) H[c * 4 + a] = f * h[a];
        }
    }

    // ghost row of the window beyond a y side that is not periodic
    __device__ __forceinline__ void ghost(int kind, const TC (&own)[NPT], TC (&dst)[NPT]) const
    {
        const bool open = is_open(kind);
#pragma unroll
        for (int m = 0; m < NPT; ++m) dst[m] = open ? (TC)0 : own[m];
    }

    // one row: G* of row j+1 into win[HI], then finish row j
    template <int LO, int CE, int HI>
    __device__ __forceinline__ void step(int j, TC (&win)[3][NPT]) const
    {
        if (j + 1 < P->ny) xsweep(j + 1, (j + 1) & 1, win[HI]);
        else if (P->bc[3].kind == BC_PERIODIC) xsweep(0, 2, win[HI]);
        else ghost(P->bc[3].kind, win[CE], win[HI]);
        const size_t c = (size_t)j * P->nx + i;
        if (rec[c * REC + R_WALL] != 0.0) wall_row(c, j & 1, win[LO], win[CE], win[HI]);
        else finish_row(c, j & 1, win[LO], win[CE], win[HI]);
    }
};

template <typename TS, typename TC, int NPT>
__global__ __launch_bounds__(64 * WPG, (sizeof(TC) * NPT <= 32 ? 2 : 1)) void k_fused2d(const TS *__restrict__ G, TS *__restrict__ Gn,
                                                         double *__restrict__ H, const double *__restrict__ rec,
                                                         const double *__restrict__ wrec,
                                                         const Params *__restrict__ Pd, Geom geo)
{
    const Params &P = *Pd;
    __shared__ double2 s_v[64 * NPT];
    __shared__ int2 s_kl[64 * NPT];
    __shared__ double s_tab[WPG][3 * 2 * MAXV];
    for (int p = threadIdx.x; p < 64 * NPT; p += 64 * WPG) {
        const int k = p < P.nv ? p % P.nv1 : 0, l = p < P.nv ? p / P.nv1 : 0;
        s_v[p] = p < P.nv ? make_double2(P.v1_lo + (k + 0.5) * P.dv1, P.v2_lo + (l + 0.5) * P.dv2)
                          : make_double2(0.0, 0.0);
        s_kl[p] = make_int2(k, l);
    }
    __syncthreads();
    const int t = tile_of(blockIdx.x, geo.ntiles);
    if (t >= geo.ntiles) return;
    const int cg = t % geo.ncg, sg = t / geo.ncg;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: cell indices live in SGPRs
    Pass<TS, TC, NPT> ps;
    ps.G = G; ps.Gn = Gn; ps.H = H; ps.rec = rec; ps.wrec = wrec; ps.P = Pd;
    ps.sv = s_v; ps.skl = s_kl; ps.tab = s_tab[wv];
    ps.lane = threadIdx.x & 63;
    ps.i = cg * WPG + wv;
    if (ps.i >= P.nx) return;
    const int j0 = sg * geo.seg, j1 = min(P.ny, j0 + geo.seg);

    TC win[3][NPT];
    // prologue: window rows (j0 - 1, j0) in win[0], win[1]
    ps.xsweep(j0, j0 & 1, win[1]);
    if (j0 > 0) ps.xsweep(j0 - 1, 2, win[0]);
    else if (P.bc[2].kind == BC_PERIODIC) ps.xsweep(P.ny - 1, 2, win[0]);
    else ps.ghost(P.bc[2].kind, win[1], win[0]);
    int j = j0;
    for (; j + 3 <= j1; j += 3) {
        ps.template step<0, 1, 2>(j, win);
        ps.template step<1, 2, 0>(j + 1, win);
        ps.template step<2, 0, 1>(j + 2, win);
    }
    if (j < j1) ps.template step<0, 1, 2>(j, win);
    if (j + 1 < j1) ps.template step<1, 2, 0>(j + 1, win);
}

template <typename TS, typename TC>
bool launch_npt(int npt, const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                const Params *Pd, const Geom &geo, hipStream_t st)
{
    const dim3 grid(((geo.ntiles + 7) / 8) * 8), block(64 * WPG);
#define MM_CASE(N)                                                                                           \
    case N:                                                                                                  \
        hipLaunchKernelGGL((k_fused2d<TS, TC, N>), grid, block, 0, st, (const TS *)G, (TS *)Gn, H, rec, wrec, \
                           Pd, geo);                                                                          \
        return true;
    switch (npt) {
        MM_CASE(1)
        MM_CASE(2)
        MM_CASE(3)
        MM_CASE(4)
        MM_CASE(6)
        MM_CASE(8)
        MM_CASE(9)
        MM_CASE(12)
        MM_CASE(16)
    default:
        if constexpr (sizeof(TC) == 4) {
            switch (npt) {
                MM_CASE(24)
                MM_CASE(36)
            default:
                return false;
            }
        }
        return false;
    }
#undef MM_CASE
}

// nodes per lane of the generic kernel: up to 16 (1024 nodes) in FP64; with g in
// FP32 also 24 and 36 (up to 2304 nodes, e.g. a 48 x 48 velocity grid)
int npt_for(int nv, int precision)
{
    static const int opts[] = {1, 2, 3, 4, 6, 8, 9, 12, 16, 24, 36};
    const int need = (nv + 63) / 64;
    for (int o : opts)
        if (o >= need) return (o > 16 && precision == 0) ? 0 : o;
    return 0;
}

} // namespace

bool closure_pass_supported(const Params &P) { return lk_supported(P); }

bool launch_micro_closure2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                            const Params &P, const Params *Pd, const uint8_t *cls, hipStream_t st)
{
    return launch_micro_lk2d(G, Gn, H, rec, wrec, P, Pd, 1, cls, st);
}

bool fused_supported(const Params &P, int precision)
{
    if (lk_supported(P, precision)) return true;    // the lane-k pass takes the grid
    if (P.nv1 > MAXV || P.nv2 > MAXV) return false;
    return npt_for(P.nv, precision) != 0;
}

void launch_micro_fused2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                          const Params &P, const Params *Pd, int precision, hipStream_t st)
{
    // MM_GENERIC_FUSED (read per launch) forces the generic kernel, so that its
    // parity can be tested on shapes the lane-k kernel also covers
    if (std::getenv("MM_GENERIC_FUSED") || !launch_micro_lk2d(G, Gn, H, rec, wrec, P, Pd, precision, nullptr, st)) {
        const Geom geo = geometry(P, 2);
        const int npt = npt_for(P.nv, precision);
        if (precision == 0) launch_npt<double, double>(npt, G, Gn, H, rec, wrec, Pd, geo, st);
        else launch_npt<float, float>(npt, G, Gn, H, rec, wrec, Pd, geo, st);
    }
}

} // namespace mm
