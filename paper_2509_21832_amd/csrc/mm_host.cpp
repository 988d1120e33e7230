// mm_host.cpp -- implementation of the C ABI declared in include/mm.h:
// configuration checks, device buffers, the per-step launch sequence and
// kernel timing.  No arithmetic of the scheme runs here.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mm.h"
#include "mm_closure.h"
#include "mm_launch.h"
#include "mm_mlp_impl.h"

namespace {

struct TimedLaunch {
    int which;
    hipEvent_t a, b;
};

} // namespace

struct mm_ctx {
    mm_config cfg;
    mm::Params P;
    int ncell = 0, nv = 0, ncomp = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    double *Q = nullptr, *Qs = nullptr, *H = nullptr, *rec = nullptr, *wrec = nullptr, *gmom = nullptr;
    double *Gs = nullptr;          // G* scratch of the reference (unfused) 2D pass
    mm::Params *Pd = nullptr;      // device copy of P (read by the fused pass)
    void *G[2] = {nullptr, nullptr};
    bool caller_buffers = false;   // G[0], G[1] and Q belong to the caller (cfg.dev_buffers)
    int gbytes = 8, cur = 0;
    int *flag = nullptr;
    int steps_done = 0, failed = -1;
    bool fused = false, broken = false;
    // timing
    bool timing = false;
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
    int tcount[MM_TIMING_CLASSES] = {};
    double tms[MM_TIMING_CLASSES] = {};
    // closure form (and the snapshot / feature entry points)
    bool closure = false, closure_set = false;
    int residual = 0;
    mm_mlp *net = nullptr;           // NULL with closure_set: the NSF closure
    float kn_max = 0.0f;
    float *cl_feat = nullptr, *cl_kn = nullptr, *cl_out = nullptr;
    uint8_t *cl_edge = nullptr, *cl_cls = nullptr, *cl_valid[2] = {nullptr, nullptr};
    int cl_vcur = 0;
    unsigned long long *cl_ncl = nullptr;   // closure cells, summed over steps (device)
    int *cl_snap = nullptr;                  // rows of the snapshot buffers (device)
    int *cl_list = nullptr, *cl_nlist = nullptr;   // cells to rebuild (device)
    // manufactured-solution source (mm_set_source)
    int source = MM_SOURCE_NONE;
    double src_t0 = 0.0;            // time of the state when the source was set
    int src_step0 = 0;              // steps_done at that moment
    double *msrc = nullptr;         // 2D: per-cell macro source moments [ncell][6]
};

namespace {

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return MM_EDEVICE;      \
    } while (0)

int check_cfg(const mm_config *c)
{
    if (!c) return MM_EINVAL;
    if (c->dim != 1 && c->dim != 2) return MM_EINVAL;
    if (c->nx < 2 || c->nv1 < 2) return MM_EINVAL;
    if (c->dim == 2 && (c->ny < 2 || c->nv2 < 2)) return MM_EINVAL;
    if (!(c->x_hi > c->x_lo) || !(c->v1_hi > c->v1_lo)) return MM_EINVAL;
    if (c->dim == 2 && (!(c->y_hi > c->y_lo) || !(c->v2_hi > c->v2_lo))) return MM_EINVAL;
    const double box[8] = {c->x_lo, c->x_hi, c->y_lo, c->y_hi, c->v1_lo, c->v1_hi, c->v2_lo, c->v2_hi};
    for (double b : box)
        if (!std::isfinite(b)) return MM_EINVAL;
    if (!(c->eps > 0.0) || !std::isfinite(c->eps)) return MM_EINVAL;
    if (c->dt > 0.0) {                          // a given dt replaces the CFL rule
        if (!std::isfinite(c->dt)) return MM_EINVAL;
    } else if (!(c->cfl > 0.0) || !std::isfinite(c->cfl)) {
        return MM_EINVAL;
    }
    if (c->dim == 2 && (!(c->nu >= -1.0) || !(c->nu < 1.0))) return MM_EINVAL;
    if (c->tau_model < 0 || c->tau_model > 3 || !(c->tau_coef > 0.0)) return MM_EINVAL;
    if (c->proj_mode != MM_PROJ_DISCRETE && c->proj_mode != MM_PROJ_PAPER) return MM_EINVAL;
    if (c->precision != MM_FP64 && c->precision != MM_MIXED && c->precision != MM_CLOSURE) return MM_EINVAL;
    if (c->dim == 1 && c->precision != MM_FP64) return MM_EINVAL;
    const int nside = c->dim == 2 ? 4 : 2;
    for (int s = 0; s < nside; ++s) {
        const mm_bc &b = c->bc[s];
        if (b.kind < MM_BC_EXTRAP || b.kind > MM_BC_INFLOW) return MM_EINVAL;
        if (c->dim == 1 && b.kind == MM_BC_INFLOW) return MM_EINVAL;
        if (b.kind == MM_BC_WALL && !(b.T_wall > 0.0)) return MM_EINVAL;
        if (b.kind == MM_BC_INFLOW && (!(b.rho > 0.0) || !(b.T > 0.0))) return MM_EINVAL;
    }
    if ((c->bc[0].kind == MM_BC_PERIODIC) != (c->bc[1].kind == MM_BC_PERIODIC)) return MM_EINVAL;
    if (c->dim == 2 && (c->bc[2].kind == MM_BC_PERIODIC) != (c->bc[3].kind == MM_BC_PERIODIC)) return MM_EINVAL;
    // cell and node counts are ints in the kernels' index arithmetic
    const double cells = (double)c->nx * (c->dim == 2 ? c->ny : 1), nodes = (double)c->nv1 * (c->dim == 2 ? c->nv2 : 1);
    if (cells > INT_MAX || nodes > INT_MAX || cells * nodes > 4.0e10) return MM_EINVAL;
    const int nbuf = (c->dev_buffers[0] != nullptr) + (c->dev_buffers[1] != nullptr) + (c->dev_buffers[2] != nullptr);
    if (nbuf != 0 && (nbuf != 3 || c->dim != 2 || c->dev_buffers[0] == c->dev_buffers[1])) return MM_EINVAL;
    return MM_OK;
}

double dt_rule(const mm_config *c)
{
    const double V1 = std::fmax(std::fabs(c->v1_lo), std::fabs(c->v1_hi));
    const double dx = (c->x_hi - c->x_lo) / c->nx;
    if (c->dim == 1) return c->cfl * dx / V1;
    const double V2 = std::fmax(std::fabs(c->v2_lo), std::fabs(c->v2_hi));
    const double dy = (c->y_hi - c->y_lo) / c->ny;
    if (c->cfl_rule == MM_CFL_SUM) return c->cfl / (V1 / dx + V2 / dy);
    return c->cfl * std::fmin(dx / V1, dy / V2);
}

// kernel parameters of a checked configuration
void build_params(const mm_config *cfg, mm::Params &P)
{
    P.nx = cfg->nx;
    P.ny = cfg->dim == 2 ? cfg->ny : 1;
    P.nv1 = cfg->nv1;
    P.nv2 = cfg->dim == 2 ? cfg->nv2 : 1;
    P.nv = P.nv1 * P.nv2;
    P.x_lo = cfg->x_lo;
    P.y_lo = cfg->y_lo;
    P.v1_lo = cfg->v1_lo;
    P.v2_lo = cfg->v2_lo;
    P.dx = (cfg->x_hi - cfg->x_lo) / cfg->nx;
    P.dy = cfg->dim == 2 ? (cfg->y_hi - cfg->y_lo) / cfg->ny : 1.0;
    P.dv1 = (cfg->v1_hi - cfg->v1_lo) / cfg->nv1;
    P.dv2 = cfg->dim == 2 ? (cfg->v2_hi - cfg->v2_lo) / cfg->nv2 : 1.0;
    P.eps = cfg->eps;
    P.dt = cfg->dt > 0.0 ? cfg->dt : dt_rule(cfg);
    P.nu = cfg->nu;
    P.tau_model = cfg->tau_model;
    P.tau_coef = cfg->tau_coef;
    P.proj_mode = cfg->proj_mode;
    P.wall_es_term = cfg->wall_es_term ? 1 : 0;
    for (int s = 0; s < 4; ++s) {
        const mm_bc &b = cfg->bc[s];
        P.bc[s].kind = (cfg->dim == 1 && s >= 2) ? mm::BC_EXTRAP : b.kind;
        P.bc[s].T_wall = b.T_wall;
        P.bc[s].u_wall = b.u_wall;
        P.bc[s].rho = b.rho;
        P.bc[s].u1 = b.u1;
        P.bc[s].u2 = b.u2;
        P.bc[s].T = b.T;
    }
}

// host-side validation of a macro state given to the library
bool state_ok(const mm_config *c, const double *q, int ncell)
{
    for (int i = 0; i < ncell; ++i) {
        if (c->dim == 1) {
            const double *s = q + 3 * (size_t)i;
            const double rho = s[0], u = s[1] / rho, T = 2.0 * s[2] / rho - u * u;
            if (!(rho > 0.0) || !(T > 0.0) || !std::isfinite(u)) return false;
        } else {
            const double *s = q + 6 * (size_t)i;
            const double rho = s[0], u1 = s[1] / rho, u2 = s[2] / rho;
            const double P11 = s[3] - s[1] * u1, P12 = s[4] - s[1] * u2, P22 = s[5] - s[2] * u2;
            const double T = 0.5 * (P11 + P22) / rho;
            const double S11 = (1.0 - c->nu) * T + c->nu * P11 / rho, S22 = (1.0 - c->nu) * T + c->nu * P22 / rho;
            const double S12 = c->nu * P12 / rho;
            const double det = S11 * S22 - S12 * S12;
            if (!(rho > 0.0) || !(T > 0.0) || !(P11 > 0.0) || !(P22 > 0.0) || !(det > 0.0) ||
                !std::isfinite(u1) || !std::isfinite(u2) || !std::isfinite(P12))
                return false;
            const double dv1 = (c->v1_hi - c->v1_lo) / c->nv1, dv2 = (c->v2_hi - c->v2_lo) / c->nv2;
            if (!mm::exp_range_ok(c->v1_lo, dv1, c->nv1, c->v2_lo, dv2, c->nv2, u1, u2, 1.0 / (2.0 * T),
                                  S22 / (2.0 * det), -S12 / (2.0 * det), S11 / (2.0 * det)))
                return false;
        }
    }
    return true;
}

void release(mm_ctx *c)
{
    if (!c) return;
    if (c->st) hipStreamSynchronize(c->st);
    for (auto &t : c->pending) {
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    for (hipEvent_t e : c->pool) hipEventDestroy(e);
    double *bufs[] = {c->caller_buffers ? nullptr : c->Q, c->Qs, c->H, c->rec, c->wrec, c->gmom, c->Gs, c->msrc};
    for (double *b : bufs)
        if (b) hipFree(b);
    void *cbufs[] = {c->cl_feat, c->cl_kn, c->cl_out, c->cl_edge, c->cl_cls, c->cl_valid[0], c->cl_valid[1],
                     c->cl_ncl, c->cl_snap, c->cl_list, c->cl_nlist};
    for (void *b : cbufs)
        if (b) hipFree(b);
    if (!c->caller_buffers)
        for (void *g : c->G)
            if (g) hipFree(g);
    if (c->flag) hipFree(c->flag);
    if (c->Pd) hipFree(c->Pd);
    if (c->own_stream && c->st) hipStreamDestroy(c->st);
    delete c;
}

// the bookkeeping of a new state that is already in the device buffers
int reset_state(mm_ctx *c)
{
    const int none = INT_MAX;
    HIP_TRY(hipMemcpyAsync(c->flag, &none, sizeof(int), hipMemcpyHostToDevice, c->st));
    // closure form: the given G is current everywhere
    for (uint8_t *v : c->cl_valid)
        if (v) HIP_TRY(hipMemsetAsync(v, 1, c->ncell, c->st));
    HIP_TRY(hipMemsetAsync(c->H, 0, sizeof(double) * 4 * c->ncell, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    c->failed = -1;
    return MM_OK;
}

int upload_state(mm_ctx *c, const double *q, const double *g)
{
    HIP_TRY(hipMemcpyAsync(c->Q, q, sizeof(double) * c->ncomp * c->ncell, hipMemcpyHostToDevice, c->st));
    const size_t n = (size_t)c->ncell * c->nv;
    if (!g) {
        HIP_TRY(hipMemsetAsync(c->G[c->cur], 0, n * c->gbytes, c->st));
    } else if (c->gbytes == 8) {
        HIP_TRY(hipMemcpyAsync(c->G[c->cur], g, n * 8, hipMemcpyHostToDevice, c->st));
    } else {
        std::vector<float> tmp(n);
        for (size_t i = 0; i < n; ++i) tmp[i] = (float)g[i];
        HIP_TRY(hipMemcpyAsync(c->G[c->cur], tmp.data(), n * 4, hipMemcpyHostToDevice, c->st));
        HIP_TRY(hipStreamSynchronize(c->st));
    }
    return reset_state(c);
}

// feature / class buffers of the closure form and of the snapshot entry points
int ensure_closure_buffers(mm_ctx *c, bool stepping)
{
    const size_t n = c->ncell;
    bool ok = true;
    if (!c->cl_feat) ok = ok && hipMalloc(&c->cl_feat, sizeof(float) * mm::closure::NF * n) == hipSuccess;
    if (!c->cl_kn) ok = ok && hipMalloc(&c->cl_kn, sizeof(float) * n) == hipSuccess;
    if (!c->cl_edge) ok = ok && hipMalloc(&c->cl_edge, n) == hipSuccess;
    if (!c->cl_out) ok = ok && hipMalloc(&c->cl_out, sizeof(float) * mm::closure::NO * n) == hipSuccess;
    if (!c->cl_ncl) {
        ok = ok && hipMalloc(&c->cl_ncl, sizeof(unsigned long long)) == hipSuccess;
        if (ok) ok = hipMemset(c->cl_ncl, 0, sizeof(unsigned long long)) == hipSuccess;
    }
    if (!c->cl_snap) ok = ok && hipMalloc(&c->cl_snap, sizeof(int)) == hipSuccess;
    if (!c->cl_list) ok = ok && hipMalloc(&c->cl_list, sizeof(int) * n) == hipSuccess;
    if (!c->cl_nlist) ok = ok && hipMalloc(&c->cl_nlist, sizeof(int)) == hipSuccess;
    if (stepping) {
        if (!c->cl_cls) {
            ok = ok && hipMalloc(&c->cl_cls, n) == hipSuccess;
            if (ok) ok = hipMemset(c->cl_cls, 1, n) == hipSuccess;
        }
        for (uint8_t *&v : c->cl_valid)
            if (!v) {
                ok = ok && hipMalloc(&v, n) == hipSuccess;
                if (ok) ok = hipMemset(v, 1, n) == hipSuccess;
            }
    }
    if (!ok) {
        hipGetLastError();
        return MM_ENOMEM;
    }
    return MM_OK;
}

hipEvent_t get_event(mm_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timer {
    mm_ctx *c;
    int which;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(mm_ctx *c_, int w) : c(c_), which(w)
    {
        if (!c->timing) return;
        a = get_event(c);
        b = get_event(c);
        if (a) hipEventRecord(a, c->st);
    }
    ~Timer()
    {
        if (!c->timing || !a || !b) return;
        hipEventRecord(b, c->st);
        c->pending.push_back({which, a, b});
    }
};

void collect_timing(mm_ctx *c)
{
    for (auto &t : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            c->tcount[t.which] += 1;
            c->tms[t.which] += ms;
        }
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->pending.clear();
}

int enqueue_steps(mm_ctx *c, int nsteps)
{
    const mm::Params &P = c->P;
    if (c->closure && !c->closure_set) return MM_EINVAL;
    for (int s = 0; s < nsteps; ++s) {
        const int step = c->steps_done;
        // time t^n of the old level, for the manufactured-solution source
        const double tn = c->src_t0 + (step - c->src_step0) * P.dt;
        if (c->cfg.dim == 1) {
            void *Gn = c->G[1 - c->cur];
            {
                Timer t(c, 0);
                mm::launch_step1d(c->Q, c->Qs, (const double *)c->G[c->cur], (double *)Gn, c->H, c->flag, step, P, c->st,
                                  c->source, tn);
            }
            std::swap(c->Q, c->Qs);
        } else {
            {
                Timer t(c, 1);
                mm::launch_prep2d(c->Q, c->rec, c->wrec, c->flag, step, P, c->st);
            }
            if (c->closure) {
                {
                    Timer t(c, 4);
                    const mm::closure::MlpDev wv = c->net ? c->net->view() : mm::closure::MlpDev{};
                    mm::closure::launch_cells2d(c->Q, P, c->net ? &wv : nullptr, c->residual, c->kn_max, c->cl_cls,
                                                c->cl_out, c->H, c->cl_ncl, c->cl_nlist, c->st);
                    mm::closure::launch_rebuild2d(c->G[c->cur], c->gbytes, c->rec, c->cl_out, c->cl_cls,
                                                  c->cl_valid[c->cl_vcur], c->cl_valid[1 - c->cl_vcur], c->cl_list,
                                                  c->cl_nlist, P, c->st);
                }
                {
                    Timer t(c, 0);
                    mm::launch_micro_closure2d(c->G[c->cur], c->G[1 - c->cur], c->H, c->rec, c->wrec, P, c->Pd,
                                               c->cl_cls, c->st);
                }
                c->cl_vcur = 1 - c->cl_vcur;
                Timer t(c, 3);
                mm::launch_wall_relax2d(c->G[1 - c->cur], c->gbytes, c->H, c->rec, c->wrec, P, c->st);
            } else if (c->fused) {
                {
                    Timer t(c, 0);
                    mm::launch_micro_fused2d(c->G[c->cur], c->G[1 - c->cur], c->H, c->rec, c->wrec, P, c->Pd,
                                             c->cfg.precision, c->st);
                }
                Timer t(c, 3);
                mm::launch_wall_relax2d(c->G[1 - c->cur], c->gbytes, c->H, c->rec, c->wrec, P, c->st);
            } else {
                Timer t(c, 0);
                mm::launch_micro_ref2d((const double *)c->G[c->cur], c->Gs, (double *)c->G[1 - c->cur], c->H,
                                       c->rec, c->wrec, P, c->st);
            }
            if (c->source == MM_SOURCE_MMS) {
                Timer t(c, 0);
                mm::launch_source2d(c->G[1 - c->cur], c->gbytes, c->H, c->rec, c->msrc, P, tn, c->st);
            }
            {
                Timer t(c, 2);
                mm::launch_macro2d(c->Q, c->Qs, c->H, c->flag, step, P, c->st,
                                   c->source == MM_SOURCE_MMS ? c->msrc : nullptr);
            }
        }
        if (hipGetLastError() != hipSuccess) {
            c->broken = true;
            return MM_EDEVICE;
        }
        c->cur = 1 - c->cur;
        c->steps_done += 1;
    }
    return MM_OK;
}

int finish(mm_ctx *c)
{
    if (hipStreamSynchronize(c->st) != hipSuccess) {
        c->broken = true;
        return MM_EDEVICE;
    }
    collect_timing(c);
    int f = INT_MAX;
    if (hipMemcpy(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
        c->broken = true;
        return MM_EDEVICE;
    }
    if (f != INT_MAX) {
        c->failed = f;
        return MM_ENONPHYS;
    }
    return MM_OK;
}

} // namespace


// ---------------------------------------------------------------------------
// Allocation-free stepping (mm_step2d_noalloc).  Every intermediate buffer of
// the 2D step lives in one static device array per GPU, carved as
//   [Params | flag | Q half state 6N | H 4N | cell records REC N | wall records WREC N]
// with N = MM_NOALLOC_MAX_CELLS; each region starts on a 256-byte boundary.
namespace noalloc {

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t N = MM_NOALLOC_MAX_CELLS;
constexpr size_t OFF_PARAMS = 0;
constexpr size_t OFF_FLAG = align256(OFF_PARAMS + sizeof(mm::Params));
constexpr size_t OFF_QS = align256(OFF_FLAG + sizeof(int));
constexpr size_t OFF_H = align256(OFF_QS + sizeof(double) * 6 * N);
constexpr size_t OFF_REC = align256(OFF_H + sizeof(double) * 4 * N);
constexpr size_t OFF_WREC = align256(OFF_REC + sizeof(double) * mm::REC * N);
constexpr size_t BYTES = align256(OFF_WREC + sizeof(double) * mm::WREC * N);
static_assert(MM_NOALLOC_BYTES_PER_CELL == sizeof(double) * (6 + 4 + mm::REC + mm::WREC),
              "per-cell figure of the header");

constexpr int MAX_DEVICES = 64;
std::mutex lock;
void *dev_ptr[MAX_DEVICES] = {};

} // namespace noalloc

// The array itself.  In host code its name is only a stand-in for the symbol:
// kernels and copies take the device address that hipGetSymbolAddress returns
// for the current device (noalloc_base).
static __device__ __align__(256) unsigned char scratch[noalloc::BYTES];

// Parameters, flag and (optionally) H of one call, set on the device by a kernel
// so that the call records no memset or host-to-device copy.
__global__ void k_noalloc_setup(mm::Params P, mm::Params *Pd, int *flag, double *H, int nH)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *Pd = P;
        *flag = INT_MAX;
    }
    for (int i = t; i < nH; i += gridDim.x * blockDim.x) H[i] = 0.0;
}

namespace {

// device address of `scratch` on `device` (made current by the caller); looked up
// once per device and kept until the process ends
unsigned char *noalloc_base(int device)
{
    if (device < 0 || device >= noalloc::MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(noalloc::lock);
    if (!noalloc::dev_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            hipGetLastError();
            return nullptr;
        }
        noalloc::dev_ptr[device] = ptr;
    }
    return (unsigned char *)noalloc::dev_ptr[device];
}

} // namespace

extern "C" {

double mm_dt(const mm_config *cfg, double t_final, int *nsteps)
{
    if (check_cfg(cfg) != MM_OK) return -1.0;
    double dt = cfg->dt > 0.0 ? cfg->dt : dt_rule(cfg);
    if (t_final > 0.0) {
        const double steps = std::ceil(t_final / dt);
        if (!(steps <= (double)INT_MAX)) return -1.0;    // more steps than an int holds (or t_final not finite)
        const int n = (int)steps;
        dt = t_final / n;
        if (nsteps) *nsteps = n;
    } else if (nsteps) {
        *nsteps = 0;
    }
    return dt;
}

int mm_init(const mm_config *cfg, const double *q0, const double *g0, mm_ctx **out)
{
    if (!out) return MM_EINVAL;
    *out = nullptr;
    int rc = check_cfg(cfg);
    if (rc) return rc;
    const bool caller = cfg->dev_buffers[0] != nullptr;
    if (!q0 && !caller) return MM_EINVAL;
    mm_ctx *c = new (std::nothrow) mm_ctx();
    if (!c) return MM_ENOMEM;
    c->cfg = *cfg;
    c->caller_buffers = caller;
    c->ncell = cfg->nx * (cfg->dim == 2 ? cfg->ny : 1);
    c->nv = cfg->nv1 * (cfg->dim == 2 ? cfg->nv2 : 1);
    c->ncomp = cfg->dim == 2 ? 6 : 3;
    if (q0 && !state_ok(cfg, q0, c->ncell)) {
        delete c;
        return MM_ENONPHYS;
    }
    mm::Params &P = c->P;
    build_params(cfg, P);
    c->gbytes = cfg->precision == MM_FP64 ? 8 : 4;
    c->fused = cfg->dim == 2 && mm::fused_supported(P, cfg->precision) && !std::getenv("MM_REFERENCE_PASS");
    if (cfg->dim == 2 && !c->fused && cfg->precision != MM_FP64) {
        delete c;
        return MM_EINVAL;          // the FP32-storage forms exist only as the fused pass
    }
    c->closure = cfg->precision == MM_CLOSURE;
    if (c->closure && !mm::closure_pass_supported(P)) {
        delete c;
        return MM_EINVAL;          // the closure form runs on the lane-k pass only
    }
    if (hipSetDevice(cfg->device) != hipSuccess) {
        delete c;
        return MM_EDEVICE;
    }
    if (cfg->stream) {
        c->st = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return MM_EDEVICE;
        }
        c->own_stream = true;
    }
    const size_t ncell = c->ncell, npts = ncell * c->nv;
    bool ok = hipMalloc(&c->Qs, sizeof(double) * c->ncomp * ncell) == hipSuccess &&
              hipMalloc(&c->H, sizeof(double) * 4 * ncell) == hipSuccess &&
              hipMalloc(&c->flag, sizeof(int)) == hipSuccess;
    if (caller) {
        c->G[0] = cfg->dev_buffers[0];
        c->G[1] = cfg->dev_buffers[1];
        c->Q = (double *)cfg->dev_buffers[2];
    } else {
        ok = ok && hipMalloc(&c->Q, sizeof(double) * c->ncomp * ncell) == hipSuccess &&
             hipMalloc(&c->G[0], npts * c->gbytes) == hipSuccess &&
             hipMalloc(&c->G[1], npts * c->gbytes) == hipSuccess;
    }
    if (ok && cfg->dim == 2)
        ok = hipMalloc(&c->rec, sizeof(double) * mm::REC * ncell) == hipSuccess &&
             hipMalloc(&c->wrec, sizeof(double) * mm::WREC * ncell) == hipSuccess;
    if (ok && cfg->dim == 2 && !c->fused) ok = hipMalloc(&c->Gs, sizeof(double) * npts) == hipSuccess;
    if (ok && c->fused) ok = hipMalloc(&c->Pd, sizeof(mm::Params)) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        release(c);
        return MM_ENOMEM;
    }
    if (c->closure && ensure_closure_buffers(c, true) != MM_OK) {
        release(c);
        return MM_ENOMEM;
    }
    if (c->Pd && hipMemcpy(c->Pd, &c->P, sizeof(mm::Params), hipMemcpyHostToDevice) != hipSuccess) {
        release(c);
        return MM_EDEVICE;
    }
    rc = q0 ? upload_state(c, q0, g0) : reset_state(c);
    if (rc) {
        release(c);
        return rc;
    }
    *out = c;
    return MM_OK;
}

int mm_step_async(mm_ctx *ctx, int nsteps)
{
    if (!ctx || nsteps < 0) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) return MM_EDEVICE;
    return enqueue_steps(ctx, nsteps);
}

int mm_sync(mm_ctx *ctx)
{
    if (!ctx) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    return finish(ctx);
}

int mm_step(mm_ctx *ctx, int nsteps)
{
    int rc = mm_step_async(ctx, nsteps);
    if (rc) return rc;
    return finish(ctx);
}

int mm_moments(mm_ctx *ctx, double *q_out, double *h_out, double *gmom_out)
{
    if (!ctx || !q_out) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (gmom_out && ctx->cfg.dim != 2) return MM_EINVAL;
    if (gmom_out) {
        if (!ctx->gmom && hipMalloc(&ctx->gmom, sizeof(double) * 7 * ctx->ncell) != hipSuccess) return MM_ENOMEM;
        // cell velocities of the current state for the centred moments
        mm::launch_prep2d(ctx->Q, ctx->rec, ctx->wrec, ctx->flag, ctx->steps_done, ctx->P, ctx->st);
        mm::launch_gmom2d(ctx->G[ctx->cur], ctx->gbytes, ctx->rec, ctx->gmom, ctx->P, ctx->st);
    }
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    HIP_TRY(hipMemcpy(q_out, ctx->Q, sizeof(double) * ctx->ncomp * ctx->ncell, hipMemcpyDeviceToHost));
    if (h_out) {
        if (ctx->cfg.dim == 2) {
            HIP_TRY(hipMemcpy(h_out, ctx->H, sizeof(double) * 4 * ctx->ncell, hipMemcpyDeviceToHost));
        } else {
            HIP_TRY(hipMemcpy(h_out, ctx->H, sizeof(double) * ctx->ncell, hipMemcpyDeviceToHost));
        }
    }
    if (gmom_out) HIP_TRY(hipMemcpy(gmom_out, ctx->gmom, sizeof(double) * 7 * ctx->ncell, hipMemcpyDeviceToHost));
    return MM_OK;
}

int mm_get_g(mm_ctx *ctx, double *g_out)
{
    if (!ctx || !g_out) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    const size_t n = (size_t)ctx->ncell * ctx->nv;
    if (ctx->gbytes == 8) {
        HIP_TRY(hipMemcpy(g_out, ctx->G[ctx->cur], n * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(n);
        HIP_TRY(hipMemcpy(tmp.data(), ctx->G[ctx->cur], n * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < n; ++i) g_out[i] = tmp[i];
    }
    return MM_OK;
}

int mm_get_g_cells(mm_ctx *ctx, const int *cells, int n, double *g_out)
{
    if (!ctx || n < 0 || (n > 0 && (!cells || !g_out))) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    for (int t = 0; t < n; ++t)
        if (cells[t] < 0 || cells[t] >= ctx->ncell) return MM_EINVAL;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    const size_t nv = (size_t)ctx->nv;
    std::vector<float> tmp(ctx->gbytes == 4 ? nv : 0);
    for (int t = 0; t < n; ++t) {
        const char *src = (const char *)ctx->G[ctx->cur] + (size_t)cells[t] * nv * ctx->gbytes;
        double *dst = g_out + (size_t)t * nv;
        if (ctx->gbytes == 8) {
            HIP_TRY(hipMemcpy(dst, src, nv * 8, hipMemcpyDeviceToHost));
        } else {
            HIP_TRY(hipMemcpy(tmp.data(), src, nv * 4, hipMemcpyDeviceToHost));
            for (size_t p = 0; p < nv; ++p) dst[p] = tmp[p];
        }
    }
    return MM_OK;
}

int mm_set_state(mm_ctx *ctx, const double *q, const double *g)
{
    if (!ctx || !q) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (!state_ok(&ctx->cfg, q, ctx->ncell)) return MM_ENONPHYS;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    return upload_state(ctx, q, g);
}

void mm_free(mm_ctx *ctx) { release(ctx); }

int mm_failed_step(const mm_ctx *ctx) { return ctx ? ctx->failed : -1; }

int mm_set_source(mm_ctx *ctx, int kind, double t0)
{
    if (!ctx || (kind != MM_SOURCE_NONE && kind != MM_SOURCE_MMS) || !std::isfinite(t0)) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (kind == MM_SOURCE_MMS && ctx->closure) return MM_EINVAL;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) return MM_EDEVICE;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    if (kind == MM_SOURCE_MMS && ctx->cfg.dim == 2 && !ctx->msrc) {
        if (hipMalloc(&ctx->msrc, sizeof(double) * 6 * ctx->ncell) != hipSuccess) {
            hipGetLastError();
            ctx->msrc = nullptr;
            return MM_ENOMEM;
        }
    }
    ctx->source = kind;
    ctx->src_t0 = t0;
    ctx->src_step0 = ctx->steps_done;
    return MM_OK;
}

const char *mm_strerror(int status)
{
    switch (status) {
    case MM_OK: return "ok";
    case MM_EINVAL: return "invalid configuration or argument";
    case MM_ENOMEM: return "out of memory";
    case MM_EDEVICE: return "HIP runtime error";
    case MM_ENONPHYS:
        return "non-physical macro state (rho, T or det of the ES temperature tensor not positive, or not finite; "
               "or, in 2D, a Maxwellian exponent beyond 600 on the velocity grid)";
    case MM_ESTATE: return "context unusable after an earlier device error";
    default: return "unknown status";
    }
}

int mm_timing(mm_ctx *ctx, int enable)
{
    if (!ctx) return MM_EINVAL;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    collect_timing(ctx);
    ctx->timing = enable != 0;
    for (int w = 0; w < MM_TIMING_CLASSES; ++w) {
        ctx->tcount[w] = 0;
        ctx->tms[w] = 0.0;
    }
    return MM_OK;
}

int mm_timing_get(mm_ctx *ctx, int which, int *count, double *total_ms)
{
    if (!ctx || which < 0 || which >= MM_TIMING_CLASSES) return MM_EINVAL;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    collect_timing(ctx);
    if (count) *count = ctx->tcount[which];
    if (total_ms) *total_ms = ctx->tms[which];
    return MM_OK;
}

int mm_device_ptrs(mm_ctx *ctx, void **q, void **g, void **h, int *g_bytes)
{
    if (!ctx) return MM_EINVAL;
    if (q) *q = ctx->Q;
    if (g) *g = ctx->G[ctx->cur];
    if (h) *h = ctx->H;
    if (g_bytes) *g_bytes = ctx->gbytes;
    return MM_OK;
}

int mm_closure_attach(mm_ctx *ctx, mm_mlp *net, double kn_max, int residual)
{
    if (!ctx || !ctx->closure || !(kn_max >= 0.0) || residual < 0 || residual > 2) return MM_EINVAL;
    if (net && net->device != ctx->cfg.device) return MM_EINVAL;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    ctx->net = net;
    ctx->residual = residual;
    ctx->kn_max = (float)kn_max;
    ctx->closure_set = true;
    return MM_OK;
}

int mm_closure_cells(mm_ctx *ctx, long long *n_closure, unsigned char *cls_host)
{
    if (!ctx || !ctx->closure) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    if (n_closure) {
        unsigned long long v = 0;
        HIP_TRY(hipMemcpy(&v, ctx->cl_ncl, sizeof(v), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemset(ctx->cl_ncl, 0, sizeof(v)));
        *n_closure = (long long)v;
    }
    if (cls_host) HIP_TRY(hipMemcpy(cls_host, ctx->cl_cls, ctx->ncell, hipMemcpyDeviceToHost));
    return MM_OK;
}

int mm_closure_snapshot(mm_ctx *ctx, double kn_max, int residual, float *x_dev, float *y_dev, int capacity,
                        int *count)
{
    if (!ctx || ctx->cfg.dim != 2 || ctx->closure || !x_dev || !y_dev || !count || *count < 0 || capacity < 0 ||
        residual < 0 || residual > 2)
        return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) return MM_EDEVICE;
    int rc = ensure_closure_buffers(ctx, false);
    if (rc) return rc;
    if (!ctx->gmom && hipMalloc(&ctx->gmom, sizeof(double) * 7 * ctx->ncell) != hipSuccess) return MM_ENOMEM;
    mm::closure::launch_features2d(ctx->Q, ctx->P, ctx->cl_feat, ctx->cl_kn, ctx->cl_edge, ctx->st);
    rc = enqueue_steps(ctx, 1);
    if (rc) return rc;
    // g-moments of G^{n+1}; the cell records still hold the velocities of Q^n
    mm::launch_gmom2d(ctx->G[ctx->cur], ctx->gbytes, ctx->rec, ctx->gmom, ctx->P, ctx->st);
    int *dcount = ctx->cl_snap;
    mm::closure::launch_snapshot2d(ctx->cl_feat, ctx->cl_kn, ctx->cl_edge, ctx->H, ctx->gmom, ctx->ncell, ctx->P,
                                   residual, (float)kn_max, x_dev, y_dev, *count, capacity, dcount, ctx->st);
    if (hipGetLastError() != hipSuccess) {
        ctx->broken = true;
        return MM_EDEVICE;
    }
    rc = finish(ctx);
    int v = 0;
    HIP_TRY(hipMemcpy(&v, dcount, sizeof(int), hipMemcpyDeviceToHost));
    *count = v;
    return rc;
}

int mm_closure_features(mm_ctx *ctx, float *feat_host, float *kn_host, unsigned char *edge_host)
{
    if (!ctx || ctx->cfg.dim != 2 || !feat_host) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) return MM_EDEVICE;
    int rc = ensure_closure_buffers(ctx, false);
    if (rc) return rc;
    mm::closure::launch_features2d(ctx->Q, ctx->P, ctx->cl_feat, ctx->cl_kn, ctx->cl_edge, ctx->st);
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    const size_t n = ctx->ncell;
    HIP_TRY(hipMemcpy(feat_host, ctx->cl_feat, sizeof(float) * mm::closure::NF * n, hipMemcpyDeviceToHost));
    if (kn_host) HIP_TRY(hipMemcpy(kn_host, ctx->cl_kn, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (edge_host) HIP_TRY(hipMemcpy(edge_host, ctx->cl_edge, n, hipMemcpyDeviceToHost));
    return MM_OK;
}

int mm_closure_rebuild(mm_ctx *ctx, const float *out_host, const unsigned char *mask)
{
    if (!ctx || ctx->cfg.dim != 2 || ctx->cfg.precision == MM_FP64 || !out_host || !mask) return MM_EINVAL;
    if (ctx->broken) return MM_ESTATE;
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) return MM_EDEVICE;
    int rc = ensure_closure_buffers(ctx, false);
    if (rc) return rc;
    // the uploads below go through the null stream, which does not wait for the
    // context's (non-blocking) stream: finish any enqueued steps first
    if (hipStreamSynchronize(ctx->st) != hipSuccess) return MM_EDEVICE;
    const size_t n = ctx->ncell;
    // classes = mask and validity = not mask: exactly the masked cells are rebuilt
    uint8_t *cls = nullptr, *valid = nullptr, *vnext = nullptr;
    if (hipMalloc(&cls, n) != hipSuccess || hipMalloc(&valid, n) != hipSuccess || hipMalloc(&vnext, n) != hipSuccess) {
        hipGetLastError();
        if (cls) hipFree(cls);
        if (valid) hipFree(valid);
        return MM_ENOMEM;
    }
    std::vector<uint8_t> m(n), v(n);
    for (size_t k = 0; k < n; ++k) {
        m[k] = mask[k] ? 1 : 0;
        v[k] = 1 - m[k];
    }
    rc = MM_OK;
    if (hipMemcpy(cls, m.data(), n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(valid, v.data(), n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->cl_out, out_host, sizeof(float) * mm::closure::NO * n, hipMemcpyHostToDevice) != hipSuccess)
        rc = MM_EDEVICE;
    if (!rc) {
        mm::launch_prep2d(ctx->Q, ctx->rec, ctx->wrec, ctx->flag, ctx->steps_done, ctx->P, ctx->st);
        if (hipMemsetAsync(ctx->cl_nlist, 0, sizeof(int), ctx->st) != hipSuccess) rc = MM_EDEVICE;
        else
            mm::closure::launch_rebuild2d(ctx->G[ctx->cur], ctx->gbytes, ctx->rec, ctx->cl_out, cls, valid, vnext,
                                          ctx->cl_list, ctx->cl_nlist, ctx->P, ctx->st);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->st) != hipSuccess) rc = MM_EDEVICE;
    }
    hipFree(cls);
    hipFree(valid);
    hipFree(vnext);
    return rc;
}

int mm_step2d_noalloc(const mm_config *cfg, double *q_dev, void *g_dev0, void *g_dev1, double *h_dev, int nsteps,
                      int *failed_step)
{
    if (failed_step) *failed_step = -1;
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (cfg->dim != 2 || (cfg->precision != MM_FP64 && cfg->precision != MM_MIXED)) return MM_EINVAL;
    if (!q_dev || !g_dev0 || !g_dev1 || g_dev0 == g_dev1 || nsteps < 0) return MM_EINVAL;
    if ((long long)cfg->nx * cfg->ny > MM_NOALLOC_MAX_CELLS) return MM_EINVAL;
    mm::Params P;
    build_params(cfg, P);
    if (!mm::fused_supported(P, cfg->precision)) return MM_EINVAL;
    if (hipSetDevice(cfg->device) != hipSuccess) return MM_EDEVICE;
    unsigned char *base = noalloc_base(cfg->device);
    if (!base) return MM_EDEVICE;
    mm::Params *Pd = (mm::Params *)(base + noalloc::OFF_PARAMS);
    int *flag = (int *)(base + noalloc::OFF_FLAG);
    double *Qs = (double *)(base + noalloc::OFF_QS);
    double *H = h_dev ? h_dev : (double *)(base + noalloc::OFF_H);
    double *rec = (double *)(base + noalloc::OFF_REC);
    double *wrec = (double *)(base + noalloc::OFF_WREC);
    hipStream_t st = (hipStream_t)cfg->stream;
    const int ncell = cfg->nx * cfg->ny;
    hipLaunchKernelGGL(k_noalloc_setup, dim3((4 * ncell + 255) / 256), dim3(256), 0, st, P, Pd, flag, H, 4 * ncell);
    void *G[2] = {g_dev0, g_dev1};
    int cur = 0;
    for (int s = 0; s < nsteps; ++s) {
        mm::launch_prep2d(q_dev, rec, wrec, flag, s, P, st);
        mm::launch_micro_fused2d(G[cur], G[1 - cur], H, rec, wrec, P, Pd, cfg->precision, st);
        mm::launch_wall_relax2d(G[1 - cur], cfg->precision == MM_FP64 ? 8 : 4, H, rec, wrec, P, st);
        mm::launch_macro2d(q_dev, Qs, H, flag, s, P, st);
        cur = 1 - cur;
    }
    if (hipGetLastError() != hipSuccess) return MM_EDEVICE;
    if (!failed_step) return MM_OK;                 // enqueued only
    if (hipStreamSynchronize(st) != hipSuccess) return MM_EDEVICE;
    int f = INT_MAX;
    if (hipMemcpy(&f, flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return MM_EDEVICE;
    if (f != INT_MAX) {
        *failed_step = f;
        return MM_ENONPHYS;
    }
    return MM_OK;
}

} // extern "C"
