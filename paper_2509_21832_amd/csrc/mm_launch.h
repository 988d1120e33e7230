// mm_launch.h -- host-side launchers of the library's kernels (internal).
#pragma once
#include "mm_internal.h"

namespace mm {

// 2D
void launch_prep2d(const double *Q, double *rec, double *wrec, int *flag, int step, const Params &P, hipStream_t st);
void launch_micro_ref2d(const double *G, double *Gs, double *Gn, double *H, const double *rec, const double *wrec,
                        const Params &P, hipStream_t st);
// msrc: nullptr, or per-cell source moments [ncell][6] added (times dt) between the
// y-sweep and the second collision half step
void launch_macro2d(double *Q, double *Qs, const double *H, int *flag, int step, const Params &P, hipStream_t st,
                    const double *msrc = nullptr);
// manufactured-solution source of the 2D convergence study at time t (mm_source.hip):
// adds (rb / tau)(I - Pi)[S] to Gn and its part to H, writes the macro source moments
void launch_source2d(void *Gn, int g_bytes, double *H, const double *rec, double *msrc, const Params &P, double t,
                     hipStream_t st);
void launch_gmom2d(const void *G, int g_bytes, const double *rec, double *out, const Params &P, hipStream_t st);

// wall-adjacent cells after a fused pass (Gn holds G** there)
void launch_wall_relax2d(void *Gn, int g_bytes, double *H, const double *rec, const double *wrec, const Params &P,
                         hipStream_t st);
// the same for velocity grids of the lane-k layout; false (nothing launched) otherwise
bool launch_wall_lk2d(void *Gn, int g_bytes, double *H, const double *rec, const double *wrec, const Params &P,
                      hipStream_t st);

// fused phase-space pass; false when the shape is not supported.  Wall-adjacent
// cells leave it holding G** and are finished by launch_wall_relax2d.
bool fused_supported(const Params &P, int precision);
// P: host copy of the parameters; Pd: the same parameters in device memory
void launch_micro_fused2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                          const Params &P, const Params *Pd, int precision, hipStream_t st);

// closure form (g in FP32): the fused pass on the cells flagged in cls only
// (and the G* rows their y-sweep needs); shapes of the lane-k kernel only
bool closure_pass_supported(const Params &P);
bool launch_micro_closure2d(const void *G, void *Gn, double *H, const double *rec, const double *wrec,
                            const Params &P, const Params *Pd, const uint8_t *cls, hipStream_t st);

// 1D
// mms != 0: with the manufactured-solution source of the 1D convergence study at time t
void launch_step1d(const double *Q, double *Qn, const double *G, double *Gn, double *H, int *flag, int step,
                   const Params &P, hipStream_t st, int mms = 0, double t = 0.0);

} // namespace mm
