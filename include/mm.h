/*
 * mm.h -- C ABI of the MI355X (gfx950) micro-macro KFVS solver for the
 * Boltzmann-BGK (1D1V) and Boltzmann-ES-BGK (2D2V) equations of
 * J.A. Rossmanith and P. Sar, "Micro-macro kinetic flux-vector splitting
 * schemes for the multidimensional Boltzmann-ES-BGK equation",
 * arXiv:2509.21832.
 *
 * One time step is the paper's micro step followed by its macro step:
 *   2D (Sec. 5.3-5.4): G^n -x-transport-> G* -y-transport-> G**
 *       -backward-Euler relaxation to G-hat (eqn5-97, eqn5-98)-> G^{n+1};
 *       H^{n+1} = eps dv sum w^3 G^{n+1} (eqn5-99);
 *       Q^n -TR-BDF2 half step-> Q* -KFVS x + dH/dx-> Q** -KFVS y + dH/dy->
 *       Q*** -TR-BDF2 half step-> Q^{n+1} (macro2d-split1..4, eqn5-103).
 *   1D (Sec. 3.3-3.4): eqn5-19 .. eqn5-25 (micro), eqn5-26, eqn5-27 (macro).
 * Every step runs on the GPU; the host only enqueues kernels.
 *
 * Conventions shared by all entry points
 *   - Status codes: every function returns an mm_status; nothing throws or
 *     aborts across this ABI.  mm_strerror() names a code.
 *   - Host buffers are owned by the caller and are not retained after the
 *     call returns.  Device memory and the context are owned by the library
 *     and released by mm_free().
 *   - Layouts (C order, FP64 on the host side):
 *       Q  [ny][nx][ncomp]      ncomp = 6 in 2D: (rho, rho u1, rho u2, E11, E12, E22),
 *                                E = rho u (x) u + P (Sec. 5.2); ncomp = 3 in 1D:
 *                                (rho, rho u, E), E = rho T/2 + rho u^2/2 (eq5-11).
 *       G  [ny][nx][nv2][nv1]   micro part g at the phase-space nodes, v1 fastest
 *                                (1D: [nx][nv1]).
 *       H  [ny][nx][4]          heat-flux tensor (H111, H112, H122, H222) (eqn5-99);
 *                                1D: [nx][1], H = (eps/2) dv sum v^3 G (eqn5-26).
 *   - One context is used by one host thread at a time; contexts are
 *     independent.  The library holds no global state.
 */
#ifndef MM_H
#define MM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_ctx mm_ctx;

enum mm_status {
    MM_OK = 0,
    MM_EINVAL = 1,     /* invalid configuration or argument                    */
    MM_ENOMEM = 2,     /* device or host allocation failed                     */
    MM_EDEVICE = 3,    /* a HIP runtime call failed                            */
    MM_ENONPHYS = 4,   /* rho <= 0, T <= 0, det(calT) <= 0 or a non-finite value; in 2D also a
                          Maxwellian or ES Gaussian whose exponent exceeds 600 at a node of the
                          velocity grid (a gas too cold for the grid to resolve) */
    MM_ESTATE = 5      /* the context is unusable (an earlier device error)     */
};

/* boundary kinds of one side of the spatial box */
enum {
    MM_BC_EXTRAP = 0,    /* constant extrapolation ("outflow"), Sec. 5.3.1 / 5.4.1   */
    MM_BC_PERIODIC = 1,  /* periodic, Sec. 5.3.2 / 5.4.2 (both sides of an axis)    */
    MM_BC_WALL = 2,      /* diffusely reflecting wall at T_wall, moving tangentially
                            with u_wall (the lid), Sec. 6.3; in 1D the walls of
                            Sec. 4.3 (u_wall unused)                                 */
    MM_BC_INFLOW = 3     /* fixed ghost Maxwellian (rho, u1, u2, T) entering the box;
                            wall machinery otherwise (g = 0 ghosts, H ghost = 0); 2D only */
};

/* collision parameter tau(rho, p, T) */
enum {
    MM_TAU_RHO = 0,      /* tau = coef * rho   (coef = 3 C25 pi/(2 sqrt 2), eqn:tau-for-2d-es-bgk) */
    MM_TAU_P = 1,        /* tau = coef * p     (eqn:collision_parameter_1d_p)                    */
    MM_TAU_HS1D = 2,     /* tau = coef * sqrt(T/(2 pi)) (coef = 16/5, eqn:collision_parameter_1d) */
    MM_TAU_CONST = 3     /* tau = coef                                                          */
};

/* projector onto the null space of the collision operator */
enum {
    MM_PROJ_DISCRETE = 0,  /* orthogonal projector of the midpoint quadrature (discrete
                              Gram matrix); also applied to G-hat.  Default.          */
    MM_PROJ_PAPER = 1      /* the continuous normalisation 1/rho of (coeffs-2D-xdir)
                              with midpoint sums, verbatim                           */
};

/* time-step rule: dt = cfl * min(dx/V1, dy/V2) (CFL-2D-part1) or
 * dt = cfl / (V1/dx + V2/dy) (the rule the printed cylindrical run follows) */
enum { MM_CFL_MIN = 0, MM_CFL_SUM = 1 };

/* arithmetic of the phase-space pass */
enum {
    MM_FP64 = 0,    /* everything FP64                                               */
    MM_MIXED = 1,   /* g stored and transported in FP32; velocity reductions, cell
                       coefficients, Gaussian / pressure-tensor algebra and the macro
                       update in FP64                                                 */
    MM_CLOSURE = 2  /* MM_MIXED plus the learned closure in near-continuum cells
                       (2D, velocity grids with nv1 dividing 64, nv1 nv2 a power-of-two
                       multiple of 64 up to 1024); see mm_closure_attach()             */
};

/* one side of the box: 0 = x_lo, 1 = x_hi, 2 = y_lo, 3 = y_hi */
typedef struct {
    int kind;
    double T_wall;          /* MM_BC_WALL: wall temperature (> 0)                 */
    double u_wall;          /* MM_BC_WALL: wall speed tangential to the side      */
    double rho, u1, u2, T;  /* MM_BC_INFLOW: ghost state                          */
} mm_bc;

typedef struct {
    int dim;                          /* 1 (1D1V) or 2 (2D2V)                       */
    int nx, ny, nv1, nv2;             /* cells / velocity nodes; ny = nv2 = 1 in 1D  */
    double x_lo, x_hi, y_lo, y_hi;    /* spatial box (cell-centred uniform grid)    */
    double v1_lo, v1_hi, v2_lo, v2_hi;/* velocity box (midpoint nodes)              */
    double eps;                       /* Knudsen number, > 0                        */
    double cfl;                       /* > 0                                        */
    int cfl_rule;                     /* MM_CFL_MIN | MM_CFL_SUM                    */
    double nu;                        /* ES-BGK parameter, -1 <= nu < 1 (2D); unused in 1D */
    int tau_model;                    /* MM_TAU_*                                   */
    double tau_coef;
    mm_bc bc[4];
    int proj_mode;                    /* MM_PROJ_*                                  */
    int wall_es_term;                 /* keep (G - M)/eps in wall-cell G-hat (1 = yes) */
    double dt;                        /* > 0: use this dt instead of the CFL rule   */
    int precision;                    /* MM_FP64 | MM_MIXED | MM_CLOSURE            */
    int device;                       /* HIP device ordinal                         */
    void *stream;                     /* hipStream_t to enqueue on; NULL: the library
                                         creates its own (default-priority) stream  */
    void *dev_buffers[3];             /* 2D only, optional: caller-owned device buffers
                                         G0, G1 (each [ny][nx][nv2][nv1], FP64 for
                                         MM_FP64, FP32 otherwise) and Q ([ny][nx][6]
                                         FP64), used instead of library allocations
                                         (zero-copy state, e.g. torch tensors); all
                                         three or none.  They must outlive the context,
                                         which never frees them.  G^n is in G0 after an
                                         even and in G1 after an odd number of steps
                                         (mm_device_ptrs names the current one). */
} mm_config;

/*
 * mm_init -- validate cfg, allocate device state, upload the initial data.
 *   q0: host Q^0 (layout above); required, except with cfg->dev_buffers, where
 *       NULL means that Q^0 and G^0 are already in the Q and G0 buffers (taken
 *       as they are: the state is checked by the first step, not here).
 *   g0: host G^0 (layout above) or NULL for g = 0, the paper's initial
 *       condition in every example (with q0 != NULL).
 *   *out receives the context, or NULL on failure (nothing leaks).
 * Errors: MM_EINVAL (bad sizes: more than INT_MAX cells or velocity nodes, or
 * more than 4e10 phase-space points; non-finite box bounds, eps, cfl or dt;
 * eps <= 0, cfl <= 0 without dt, nu outside [-1, 1) in 2D,
 * unpaired periodic sides, inflow sides in 1D, T_wall <= 0, dev_buffers partly set, set
 * in 1D or with two equal G buffers), MM_ENONPHYS (Q^0 not physical), MM_ENOMEM,
 * MM_EDEVICE.
 */
int mm_init(const mm_config *cfg, const double *q0, const double *g0, mm_ctx **out);

/*
 * mm_step -- advance nsteps fixed-dt steps, then wait for the GPU once.
 * Returns MM_ENONPHYS if some step produced a non-physical macro state
 * (mm_failed_step() gives the first such step, counted from the start of the
 * run); the state then holds the result of the last step enqueued.
 */
int mm_step(mm_ctx *ctx, int nsteps);

/* mm_step_async -- enqueue nsteps steps on the context's stream and return
 * without waiting; the non-physical check happens at the next mm_sync(). */
int mm_step_async(mm_ctx *ctx, int nsteps);

/* mm_sync -- wait for the stream; returns MM_ENONPHYS as mm_step would. */
int mm_sync(mm_ctx *ctx);

/*
 * mm_moments -- wait for the stream and copy the macro state out.
 *   q_out  host Q (required)            [ny][nx][ncomp]
 *   h_out  host H of the last step or NULL  [ny][nx][4] (1D: [nx])
 *   gmom_out host g-moments or NULL     [ny][nx][7] (2D only):
 *          dv sum (1, v1, v2, |v|^2/2) G (zero up to round-off with the discrete
 *          projector), then eps dv sum (w1^2 - w2^2, 2 w1 w2, |w|^2) G / 2
 *          (stress deviation and trace of the micro part)
 */
int mm_moments(mm_ctx *ctx, double *q_out, double *h_out, double *gmom_out);

/* mm_get_g -- copy G out as FP64 (host [ny][nx][nv2][nv1]). */
int mm_get_g(mm_ctx *ctx, double *g_out);

/* mm_get_g_cells -- copy G of n cells out as FP64: cells[t] is the cell index
 * j * nx + i (host, 0 <= cells[t] < nx * ny), g_out is host [n][nv2][nv1].
 * MM_EINVAL for an index out of range (nothing is copied then). */
int mm_get_g_cells(mm_ctx *ctx, const int *cells, int n, double *g_out);

/* mm_set_state -- replace Q (required) and G (NULL: zero) with host data;
 * together with mm_moments/mm_get_g this is checkpoint / restart. */
int mm_set_state(mm_ctx *ctx, const double *q, const double *g);

/* mm_free -- release the context; mm_free(NULL) does nothing. */
void mm_free(mm_ctx *ctx);

/* mm_dt -- the time step cfg implies (cfg->dt if > 0, else the CFL rule).
 * With t_final > 0 the reset rule of Sec. 3.2 / (CFL-2D-part1) is applied:
 * N = ceil(t_final / dt), dt = t_final / N, and *nsteps (if not NULL) gets N.
 * Returns a negative value for an invalid configuration, or when N would not
 * fit an int. */
double mm_dt(const mm_config *cfg, double t_final, int *nsteps);

/* mm_failed_step -- first step whose macro state was non-physical, or -1. */
int mm_failed_step(const mm_ctx *ctx);

/* source terms */
enum {
    MM_SOURCE_NONE = 0,
    MM_SOURCE_MMS = 1   /* the manufactured solution of the paper's convergence study:
                           1D (Sec. 3.4): f = (e^-(v-1)^2 + 2 e^-(v+1)^2)(2 + sin 2pi(x - t));
                           2D (Sec. 6.2): f = (e^-|v-(1,1)|^2 + 2 e^-|v+(1,1)|^2)
                                              (2 - sin 2pi(t - x) cos 2pi(t - y)).
                           Its residual S = f_t + v . grad f - (tau / eps)(calG[f] - f)
                           (calG[f] = M[f] in 1D) enters each step at the old time level
                           t^n and the cell centre: (1 / tau_ij^n)(I - Pi)[S] is added to
                           G-hat, and dt times the velocity moments of S (closed form)
                           to the macro update (1D: with the flux differences, eqn5-27;
                           2D: after the y-sweep, before the second collision half
                           step).  The tau inside S is the cell's tau_i^n in 1D and
                           that of the invented state in 2D.                         */
};

/*
 * mm_set_source -- from the next step on, add the source `kind`, with the current
 * state taken to be at time t0 (t^n = t0 + n dt for the n-th following step).
 * The initial state is the caller's (e.g. the invented solution's point values
 * at the cell centres).  Not with MM_CLOSURE.  Errors: MM_EINVAL, MM_ENOMEM,
 * MM_EDEVICE, MM_ESTATE.
 */
int mm_set_source(mm_ctx *ctx, int kind, double t0);

/* mm_strerror -- static text for a status code. */
const char *mm_strerror(int status);

/*
 * Kernel timing (HIP events recorded on the context's stream around every
 * kernel launch of a step).  mm_timing(ctx, 1) enables and resets the
 * counters; mm_timing_get() returns the number of timed launches and their
 * summed duration in milliseconds for kernel class `which`:
 *   0 = phase-space (micro) pass: the fused kernel, or both sweeps of the
 *       unfused pass, or the whole 1D step,
 *   1 = per-cell preparation, 2 = macro sweeps,
 *   3 = wall-adjacent cells after a fused pass.
 *   4 = closure-form kernels (features, network, classes, rebuilt micro parts).
 * Any other `which` gives MM_EINVAL.
 */
#define MM_TIMING_CLASSES 5
int mm_timing(mm_ctx *ctx, int enable);
int mm_timing_get(mm_ctx *ctx, int which, int *count, double *total_ms);

/* mm_device_ptrs -- device addresses of the current Q, G and H buffers (for
 * zero-copy interop, e.g. wrapping them as torch tensors).  G is FP64 or FP32
 * according to cfg->precision; *g_bytes receives its element size. */
int mm_device_ptrs(mm_ctx *ctx, void **q, void **g, void **h, int *g_bytes);

/* =====================================================================
 * Learned closure (2D).  Not part of the paper; built on its macro system:
 * the macro update of Sec. 5.4 needs from the micro part only the heat-flux
 * tensor H (eq5-41).  In near-continuum cells a network predicts, from the
 * local macro state, the heat-flux vector q, the stress deviation S and the
 * traceless third moments t of eps g, and H is rebuilt from q and t:
 *   H_abc = (q_a d_bc + q_b d_ac + q_c d_ab) / 2 + (traceless part of t),
 *   H111 = 3/2 q1 + t1/4, H112 = q2/2 + t2/4, H122 = q1/2 - t1/4,
 *   H222 = 3/2 q2 - t2/4,
 * whose contraction (H111 + H122, H112 + H222) / 2 is the heat-flux vector h
 * of Sec. 6.3 and whose traceless combinations are t = (H111 - 3 H122,
 * 3 H112 - H222); t = 0 is the isotropic (Grad) form.
 *
 * Features of a cell (30, FP32): (rho, u1, u2, T, P11, P12, P22), their
 * centred x and y differences (one-sided next to a non-periodic side), the
 * local mean free path eps sqrt(T) / tau, and the second x and y differences
 * of (rho, u1, u2, T) (zero next to a non-periodic side), in that order.  Targets (7, FP32): (q1, q2, S11, S12, S22, t1, t2) / eps with
 *   q = (H111 + H122, H112 + H222) / 2,  S = eps dv sum (w w^T) g,
 *   t = (H111 - 3 H122, 3 H112 - H222).
 * Local Knudsen indicator:
 *   kn = (eps sqrt(T) / tau) max(|grad rho| / rho, |grad T| / T, |grad u|_F / sqrt(T)).
 * A step of an MM_CLOSURE context solves the micro part (as MM_MIXED) in cells
 * next to a non-periodic side and where kn > kn_max; elsewhere H comes from
 * the closure.  Micro parts of closure cells that a solved cell needs (its
 * 3 x 3 neighbourhood) are rebuilt, when not current, as
 *   g = M / (2 p T) [S' : w w^T + (q . w)(|w|^2 / (2T) - 2)]
 *       + M / (24 p T^2) [t1 (w1^3 - 3 w1 w2^2) + t2 (3 w1^2 w2 - w2^3)],
 * then (I - Pi) g (S' the traceless part of S), which under M has exactly the
 * moments q, S, t.
 * G of closure cells is not kept current: mm_get_g and the g-moments of
 * mm_moments are meaningful only in solved cells.
 * ===================================================================== */

/* the network: 30 -> 64 -> 64 -> 7, GELU (erf form), bf16 weights and
 * activations on the matrix cores with FP32 accumulation, FP32 master weights */
typedef struct mm_mlp mm_mlp;
#define MM_MLP_NPARAM 6599   /* W1[64][30], b1[64], W2[64][64], b2[64], W3[7][64], b3[7] */
#define MM_MLP_NNORM 74      /* in_mean[30], in_std[30], out_mean[7], out_std[7]         */

/* mm_mlp_create -- a network on `device` with Glorot-uniform weights drawn
 * from `seed` (SplitMix64), zero biases and identity normalisation; stream as
 * in mm_config.  Every mm_mlp_* call returns when its work is done. */
int mm_mlp_create(int device, void *stream, unsigned long long seed, mm_mlp **out);
void mm_mlp_free(mm_mlp *net);

/* mm_mlp_fit_norm -- set the normalisation to the mean and standard deviation
 * of the n rows of x_dev [n][30] and y_dev [n][7] (device FP32). */
int mm_mlp_fit_norm(mm_mlp *net, const float *x_dev, const float *y_dev, int n);

/* mm_mlp_get / mm_mlp_set -- FP32 parameters [MM_MLP_NPARAM] and normalisation
 * [MM_MLP_NNORM] (host; either may be NULL).  mm_mlp_set resets the Adam state;
 * a standard deviation <= 0 gives MM_EINVAL. */
int mm_mlp_get(mm_mlp *net, float *params, float *norm);
int mm_mlp_set(mm_mlp *net, const float *params, const float *norm);

/* mm_mlp_forward -- raw outputs y_dev [n][7] of raw features x_dev [n][30]:
 * y = MLP((x - in_mean) / in_std) * out_std + out_mean (device FP32). */
int mm_mlp_forward(mm_mlp *net, const float *x_dev, int n, float *y_dev);

/* mm_mlp_grad -- gradient (host FP32 [MM_MLP_NPARAM], parameter order above)
 * and value (host) of L = mean over the n samples and 7 outputs of
 * (MLP(xn) - (y - out_mean) / out_std)^2; no parameter changes. */
int mm_mlp_grad(mm_mlp *net, const float *x_dev, const float *y_dev, int n, float *grad, double *loss);

/* mm_mlp_train -- `epochs` passes of Adam (beta = 0.9, 0.999; step size lr with
 * cosine decay to 0.05 lr) over mini-batches of `batch` samples (>= 32) in an
 * order drawn per epoch from `seed`; epoch_loss (host [epochs] or NULL)
 * receives the mean batch loss of each epoch. */
int mm_mlp_train(mm_mlp *net, const float *x_dev, const float *y_dev, int n, int epochs, int batch, double lr,
                 unsigned long long seed, double *epoch_loss);

/* mm_closure_attach -- closure of an MM_CLOSURE context, threshold kn_max >= 0:
 *   net == NULL: the Navier-Stokes-Fourier values
 *       q = -eps (2 p / tau) grad T,  S = -eps (p / tau) sigma + nu (P - p I)
 *     (sigma = grad u + grad u^T - (div u) I), the moments of the first-order
 *     micro part G-hat (eqn5-97);
 *     and t = 0 (G-hat's third moments are of the isotropic form);
 *   net, residual = 0: (q, S, t) / eps = the network's outputs;
 *   net, residual = 1: (q, S, t) / eps = the NSF values plus the network's outputs;
 *   net, residual = 2: (q, S, t) / eps = the NSF values plus eps times the
 *     network's outputs (networks trained on snapshots of the same residual
 *     kind, see mm_closure_snapshot).
 * The network is kept by pointer: it must outlive its use and not be trained
 * while the context steps.  Stepping an MM_CLOSURE context without a closure
 * gives MM_EINVAL.  The closure values stand for a relaxed micro part: from a
 * g that is not relaxed (g = 0 at mm_init), attach with kn_max = 0 for the
 * initial layer, a few collision times eps tau (every cell with a nonzero
 * indicator is then solved; where it is zero the state is uniform and g = 0 is
 * relaxed), and attach the threshold after it; attaching again replaces the
 * previous closure. */
int mm_closure_attach(mm_ctx *ctx, mm_mlp *net, double kn_max, int residual);

/* mm_closure_cells -- number of closure cells summed over the steps since the
 * previous call, and (cls_host [ny][nx] or NULL) 1 for solved, 0 for closure
 * cells of the last step. */
int mm_closure_cells(mm_ctx *ctx, long long *n_closure, unsigned char *cls_host);

/* mm_closure_snapshot -- training data from a full micro solve (MM_FP64 or
 * MM_MIXED context): the features of the current state, one step, the targets
 * of the new micro part (residual = 1: minus the NSF values of the cell).
 * Rows of cells with kn <= kn_max that are not next to a non-periodic side are
 * appended in cell order to x_dev [capacity][30] and y_dev [capacity][7]
 * (device FP32) from row *count on; *count is updated (at most capacity rows
 * are written). */
int mm_closure_snapshot(mm_ctx *ctx, double kn_max, int residual, float *x_dev, float *y_dev, int capacity,
                        int *count);

/* mm_closure_features -- features [ny][nx][30], kn [ny][nx] and the
 * next-to-a-non-periodic-side mask [ny][nx] of the current state (host;
 * kn_host and edge_host may be NULL). */
int mm_closure_features(mm_ctx *ctx, float *feat_host, float *kn_host, unsigned char *edge_host);

/* mm_closure_rebuild -- replace the current G of the cells with mask[c] != 0
 * (host [ny][nx]) by the micro part rebuilt from out_host [ny][nx][7] =
 * (q1, q2, S11, S12, S22, t1, t2) / eps of each cell, as a closure step does. */
int mm_closure_rebuild(mm_ctx *ctx, const float *out_host, const unsigned char *mask);

/* =====================================================================
 * Stepping without allocation.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The caller
 * owns the state in device memory; every intermediate buffer of the step (the
 * per-cell records, the wall records, the macro half state, H when h_dev is
 * NULL, the non-physical flag and the device copy of the parameters) lives in
 * one static device array of the library, MM_NOALLOC_BYTES_PER_CELL bytes per
 * cell for at most MM_NOALLOC_MAX_CELLS cells (about 39 MB), which every GPU the
 * library runs this on holds until the process ends.  The call makes no
 * hipMalloc, hipFree, memset or host-to-device copy.
 * ===================================================================== */
#define MM_NOALLOC_MAX_CELLS 65536
#define MM_NOALLOC_BYTES_PER_CELL 592   /* (6 + 4 + 48 + 16) doubles */

/*
 * mm_step2d_noalloc -- nsteps steps of the 2D step, as mm_step runs them for an
 * MM_FP64 or MM_MIXED context of cfg (the fused phase-space pass: nv1 * nv2 a
 * multiple of 64, up to 1024 nodes in FP64, 2304 with g in FP32).
 *   q_dev   device Q [ny][nx][6] FP64: Q^n on entry, the result on return.
 *   g_dev0, g_dev1  two distinct device G buffers [ny][nx][nv2][nv1], FP64
 *           (MM_FP64) or FP32 (MM_MIXED); g_dev0 holds G^n on entry, and the
 *           result is in g_dev0 after an even and in g_dev1 after an odd nsteps.
 *   h_dev   device H [ny][nx][4] FP64 of the last step, or NULL (H stays in the
 *           static array).
 *   failed_step  NULL: the work is only enqueued on cfg->stream (NULL: the null
 *           stream) and the call returns; it enqueues kernel launches only, so
 *           it can be captured in a HIP graph and replayed (the first call on a
 *           device looks up the static array's address: make it outside capture).
 *           Otherwise the call waits for the stream and, as mm_step does,
 *           returns MM_ENONPHYS with *failed_step the first non-physical step,
 *           counted from 0 at the start of this call (-1 when none).
 * Calls on one GPU share its static array, which keeps the last call's contents
 * (the parameters, flag and H are set afresh by every call): calls that overlap
 * on one GPU race, whatever their streams.
 * Errors: MM_EINVAL (bad configuration, dim != 2, another precision, a velocity
 * grid the fused pass does not take, more than MM_NOALLOC_MAX_CELLS cells, NULL
 * or equal G buffers), MM_EDEVICE (HIP failure), MM_ENONPHYS.
 */
int mm_step2d_noalloc(const mm_config *cfg, double *q_dev, void *g_dev0, void *g_dev1, double *h_dev, int nsteps,
                      int *failed_step);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
