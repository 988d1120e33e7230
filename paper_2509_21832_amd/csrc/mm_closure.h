// mm_closure.h -- the closure network's sizes, device views and the launchers
// of the closure-form kernels (internal).
#pragma once
#include <cstdint>

#include "mm_internal.h"

namespace mm {
namespace closure {

constexpr int NF = 30;      // features: (rho, u1, u2, T, P11, P12, P22), d/dx, d/dy; eps sqrt(T) / tau;
                            // d2/dx2, d2/dy2 of (rho, u1, u2, T)
static_assert(NF <= 32, "the first layer takes at most 32 inputs (two K-blocks of 16)");
constexpr int NH = 64;      // hidden width (two layers)
constexpr int NO = 7;       // outputs: (q1, q2, S11, S12, S22, t1, t2) / eps
constexpr int NPARAM = NH * NF + NH + NH * NH + NH + NO * NH + NO;   // 6599
static_assert(NO <= 8, "the output layer keeps outputs 4 g + v (g < 2, v < 4) per lane half");
constexpr int NNORM = 2 * NF + 2 * NO;   // in_mean, in_std, out_mean, out_std

// bf16 weights (W1 [64][32], W2 [64][64], W3 [32][64], zero padded, row-major:
// the training kernel), the same weights packed per lane in the operand order
// of the matrix instruction (Wp, 16 blocks of 64 lanes x 8: the inference
// path), FP32 biases and normalisation
constexpr int NWP = 16 * 64 * 8;
struct MlpDev {
    const __bf16 *W1, *W2, *W3, *Wp;
    const float *b1, *b2, *b3, *norm;
};
struct MlpDevMut {
    __bf16 *W1, *W2, *W3, *Wp;
    float *b1, *b2, *b3, *norm;
};

void launch_features2d(const double *Q, const Params &P, float *feat, float *kn, uint8_t *edge, hipStream_t st);
// the closure part of a step in one kernel: features, indicator, classes, the
// closure values out = (q, S, t) / eps (NSF, network, or NSF plus scale x network
// with residual) and H of the closure cells; empties the rebuild list
void launch_cells2d(const double *Q, const Params &P, const MlpDev *w, int residual, float kn_max, uint8_t *cls,
                    float *out, double *H, unsigned long long *nclosure, int *nrebuild, hipStream_t st);
// Y = MLP(X), or Y += scale MLP(X) with accumulate
void launch_mlp_forward(const float *X, int n, const MlpDev &w, float *Y, bool accumulate, float scale,
                        hipStream_t st);
// nwaves must be even; part holds nwaves * NPARAM floats, loss_part nwaves
void launch_mlp_grad(const float *X, const float *Y, const int *idx, int first, int count, const MlpDev &w,
                     float *part, float *loss_part, int nwaves, hipStream_t st);
void launch_mlp_reduce(const float *part, int nparts, const float *loss_part, float *grad, float *loss_acc,
                       int loss_slot, hipStream_t st);
void launch_mlp_adam(float *master, float *m1, float *m2, const float *grad, float lr, float b1, float b2, float c1,
                     float c2, float epsa, hipStream_t st);
void launch_mlp_pack(const float *master, const MlpDevMut &w, hipStream_t st);
void launch_mlp_norm(const float *X, const float *Y, int n, float *norm, hipStream_t st);
void launch_nsf2d(const float *feat, int n, const Params &P, float *out, hipStream_t st);
// classes and closure-cell H; also empties the rebuild list (*nrebuild = 0)
void launch_classify2d(const float *kn, const uint8_t *edge, const float *out, int n, float kn_max, double eps,
                       uint8_t *cls, double *H, unsigned long long *nclosure, int *nrebuild, hipStream_t st);
// list (ncell ints) the cells to rebuild, then rebuild them; *nrebuild must be 0 on entry
void launch_rebuild2d(void *G, int g_bytes, const double *rec, const float *out, const uint8_t *cls,
                      const uint8_t *valid, uint8_t *valid_next, int *list, int *nrebuild, const Params &P,
                      hipStream_t st);
void launch_snapshot2d(const float *feat, const float *kn, const uint8_t *edge, const double *H, const double *gm,
                       int n, const Params &P, int residual, float kn_max, float *Xo, float *Yo, int base,
                       int capacity, int *count, hipStream_t st);

} // namespace closure
} // namespace mm
