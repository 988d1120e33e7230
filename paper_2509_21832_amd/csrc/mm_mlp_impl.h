// mm_mlp_impl.h -- layout of the closure network object behind the opaque
// mm_mlp handle (internal; shared by mm_mlp.cpp and the solver).
#pragma once
#include <hip/hip_runtime.h>

#include "mm_closure.h"

struct mm_mlp {
    int device = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    float *master = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;   // FP32, NPARAM each
    __bf16 *W1 = nullptr, *W2 = nullptr, *W3 = nullptr, *Wp = nullptr;      // matrix-core copies
    float *b1 = nullptr, *b2 = nullptr, *b3 = nullptr, *norm = nullptr;
    float *part = nullptr, *loss_part = nullptr;   // per-wavefront partial gradients
    int nwaves_cap = 0;
    float *loss_acc = nullptr;
    int loss_cap = 0;
    int *perm = nullptr;
    int perm_cap = 0;
    long adam_t = 0;
    mm::closure::MlpDev view() const;
    mm::closure::MlpDevMut mut() const;
};
