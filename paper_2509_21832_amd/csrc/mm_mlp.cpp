// mm_mlp.cpp -- the closure network object of the C ABI (include/mm.h):
// FP32 master weights and Adam moments on the device, bf16 copies in
// matrix-core order for the kernels, normalisation statistics, and the
// training loop (mini-batch gradient on the matrix cores, fixed-order sum of
// the per-wavefront partial gradients, Adam step, re-packing).  No arithmetic
// of the network runs on the host; the host draws the initial weights and the
// per-epoch sample order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/mm.h"
#include "mm_closure.h"
#include "mm_mlp_impl.h"

static_assert(MM_MLP_NPARAM == mm::closure::NPARAM && MM_MLP_NNORM == mm::closure::NNORM,
              "parameter and normalisation sizes of the header");

using namespace mm::closure;

namespace {

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return MM_EDEVICE;      \
    } while (0)

// SplitMix64 (Steele, Lea and Flood, 2014): the generator of the initial
// weights and of the epoch permutations
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }   // [0, 1)
};

void release(mm_mlp *n)
{
    if (!n) return;
    if (n->st) hipStreamSynchronize(n->st);
    void *bufs[] = {n->master, n->m1, n->m2, n->grad, n->W1, n->W2, n->W3, n->Wp, n->b1, n->b2, n->b3, n->norm,
                    n->part, n->loss_part, n->loss_acc, n->perm};
    for (void *b : bufs)
        if (b) hipFree(b);
    if (n->own_stream && n->st) hipStreamDestroy(n->st);
    delete n;
}

int upload_params(mm_mlp *n, const float *params)
{
    HIP_TRY(hipMemcpyAsync(n->master, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, n->st));
    HIP_TRY(hipMemsetAsync(n->m1, 0, sizeof(float) * NPARAM, n->st));
    HIP_TRY(hipMemsetAsync(n->m2, 0, sizeof(float) * NPARAM, n->st));
    launch_mlp_pack(n->master, n->mut(), n->st);
    HIP_TRY(hipStreamSynchronize(n->st));
    n->adam_t = 0;
    return MM_OK;
}

// scratch of the gradient kernel for `nwaves` wavefronts
int ensure_part(mm_mlp *n, int nwaves)
{
    if (nwaves <= n->nwaves_cap) return MM_OK;
    if (n->part) hipFree(n->part);
    if (n->loss_part) hipFree(n->loss_part);
    n->part = nullptr;
    n->loss_part = nullptr;
    n->nwaves_cap = 0;
    if (hipMalloc(&n->part, sizeof(float) * NPARAM * (size_t)nwaves) != hipSuccess ||
        hipMalloc(&n->loss_part, sizeof(float) * nwaves) != hipSuccess)
        return MM_ENOMEM;
    n->nwaves_cap = nwaves;
    return MM_OK;
}

// an even number of wavefronts, about one per 32-sample tile, at most 512
int waves_for(int count)
{
    int w = (count + 31) / 32;
    if (w > 512) w = 512;
    if (w < 2) w = 2;
    return (w + 1) & ~1;
}

} // namespace

mm::closure::MlpDev mm_mlp::view() const { return {W1, W2, W3, Wp, b1, b2, b3, norm}; }
mm::closure::MlpDevMut mm_mlp::mut() const { return {W1, W2, W3, Wp, b1, b2, b3, norm}; }

extern "C" {

int mm_mlp_create(int device, void *stream, unsigned long long seed, mm_mlp **out)
{
    if (!out) return MM_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return MM_EDEVICE;
    mm_mlp *n = new (std::nothrow) mm_mlp();
    if (!n) return MM_ENOMEM;
    n->device = device;
    if (stream) {
        n->st = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&n->st, hipStreamNonBlocking) != hipSuccess) {
            delete n;
            return MM_EDEVICE;
        }
        n->own_stream = true;
    }
    bool ok = hipMalloc(&n->master, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc(&n->m1, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc(&n->m2, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc(&n->grad, sizeof(float) * NPARAM) == hipSuccess &&
              hipMalloc(&n->W1, sizeof(__bf16) * NH * 32) == hipSuccess &&
              hipMalloc(&n->W2, sizeof(__bf16) * NH * NH) == hipSuccess &&
              hipMalloc(&n->W3, sizeof(__bf16) * 32 * NH) == hipSuccess &&
              hipMalloc(&n->Wp, sizeof(__bf16) * NWP) == hipSuccess &&
              hipMalloc(&n->b1, sizeof(float) * NH) == hipSuccess &&
              hipMalloc(&n->b2, sizeof(float) * NH) == hipSuccess &&
              hipMalloc(&n->b3, sizeof(float) * NO) == hipSuccess &&
              hipMalloc(&n->norm, sizeof(float) * NNORM) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        release(n);
        return MM_ENOMEM;
    }
    // Glorot-uniform weights, zero biases; identity normalisation
    std::vector<float> p(NPARAM, 0.0f);
    SplitMix64 rng{seed};
    auto fill = [&](int off, int fan_out, int fan_in) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int t = 0; t < fan_out * fan_in; ++t) p[off + t] = (float)((2.0 * rng.uniform() - 1.0) * a);
    };
    fill(0, NH, NF);
    fill(NH * NF + NH, NH, NH);
    fill(NH * NF + NH + NH * NH + NH, NO, NH);
    std::vector<float> nrm(NNORM, 0.0f);
    for (int k = 0; k < NF; ++k) nrm[NF + k] = 1.0f;
    for (int k = 0; k < NO; ++k) nrm[2 * NF + NO + k] = 1.0f;
    if (hipMemcpy(n->norm, nrm.data(), sizeof(float) * NNORM, hipMemcpyHostToDevice) != hipSuccess ||
        upload_params(n, p.data()) != MM_OK) {
        release(n);
        return MM_EDEVICE;
    }
    *out = n;
    return MM_OK;
}

void mm_mlp_free(mm_mlp *net) { release(net); }

int mm_mlp_fit_norm(mm_mlp *n, const float *x_dev, const float *y_dev, int count)
{
    if (!n || !x_dev || !y_dev || count < 1) return MM_EINVAL;
    HIP_TRY(hipSetDevice(n->device));
    launch_mlp_norm(x_dev, y_dev, count, n->norm, n->st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(n->st));
    return MM_OK;
}

int mm_mlp_get(mm_mlp *n, float *params, float *norm)
{
    if (!n) return MM_EINVAL;
    HIP_TRY(hipSetDevice(n->device));
    HIP_TRY(hipStreamSynchronize(n->st));
    if (params) HIP_TRY(hipMemcpy(params, n->master, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (norm) HIP_TRY(hipMemcpy(norm, n->norm, sizeof(float) * NNORM, hipMemcpyDeviceToHost));
    return MM_OK;
}

int mm_mlp_set(mm_mlp *n, const float *params, const float *norm)
{
    if (!n) return MM_EINVAL;
    HIP_TRY(hipSetDevice(n->device));
    HIP_TRY(hipStreamSynchronize(n->st));
    if (norm) {
        for (int k = 0; k < NF; ++k)
            if (!(norm[NF + k] > 0.0f)) return MM_EINVAL;
        for (int k = 0; k < NO; ++k)
            if (!(norm[2 * NF + NO + k] > 0.0f)) return MM_EINVAL;
        HIP_TRY(hipMemcpy(n->norm, norm, sizeof(float) * NNORM, hipMemcpyHostToDevice));
    }
    if (params) return upload_params(n, params);
    return MM_OK;
}

int mm_mlp_forward(mm_mlp *n, const float *x_dev, int count, float *y_dev)
{
    if (!n || count < 0 || (count > 0 && (!x_dev || !y_dev))) return MM_EINVAL;
    if (count == 0) return MM_OK;
    HIP_TRY(hipSetDevice(n->device));
    launch_mlp_forward(x_dev, count, n->view(), y_dev, false, 1.0f, n->st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(n->st));
    return MM_OK;
}

int mm_mlp_grad(mm_mlp *n, const float *x_dev, const float *y_dev, int count, float *grad, double *loss)
{
    if (!n || !x_dev || !y_dev || count < 1) return MM_EINVAL;
    HIP_TRY(hipSetDevice(n->device));
    const int nw = waves_for(count);
    int rc = ensure_part(n, nw);
    if (rc) return rc;
    if (!n->loss_acc && hipMalloc(&n->loss_acc, sizeof(float) * 1) != hipSuccess) return MM_ENOMEM;
    n->loss_cap = n->loss_cap < 1 ? 1 : n->loss_cap;
    HIP_TRY(hipMemsetAsync(n->loss_acc, 0, sizeof(float), n->st));
    launch_mlp_grad(x_dev, y_dev, nullptr, 0, count, n->view(), n->part, n->loss_part, nw, n->st);
    launch_mlp_reduce(n->part, nw, n->loss_part, n->grad, n->loss_acc, 0, n->st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(n->st));
    if (grad) HIP_TRY(hipMemcpy(grad, n->grad, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (loss) {
        float l = 0.0f;
        HIP_TRY(hipMemcpy(&l, n->loss_acc, sizeof(float), hipMemcpyDeviceToHost));
        *loss = l;
    }
    return MM_OK;
}

int mm_mlp_train(mm_mlp *n, const float *x_dev, const float *y_dev, int count, int epochs, int batch, double lr,
                 unsigned long long seed, double *epoch_loss)
{
    if (!n || !x_dev || !y_dev || count < 1 || epochs < 1 || batch < 32 || !(lr > 0.0)) return MM_EINVAL;
    HIP_TRY(hipSetDevice(n->device));
    if (batch > count) batch = count < 32 ? 32 : count;
    const int nw = waves_for(batch);
    int rc = ensure_part(n, nw);
    if (rc) return rc;
    if (n->perm_cap < count) {
        if (n->perm) hipFree(n->perm);
        n->perm = nullptr;
        n->perm_cap = 0;
        if (hipMalloc(&n->perm, sizeof(int) * (size_t)count) != hipSuccess) return MM_ENOMEM;
        n->perm_cap = count;
    }
    if (n->loss_cap < epochs) {
        if (n->loss_acc) hipFree(n->loss_acc);
        n->loss_acc = nullptr;
        n->loss_cap = 0;
        if (hipMalloc(&n->loss_acc, sizeof(float) * epochs) != hipSuccess) return MM_ENOMEM;
        n->loss_cap = epochs;
    }
    HIP_TRY(hipMemsetAsync(n->loss_acc, 0, sizeof(float) * epochs, n->st));
    const int nbatch = (count + batch - 1) / batch;
    const long total = (long)nbatch * epochs;
    const float b1 = 0.9f, b2 = 0.999f, epsa = 1e-8f;
    std::vector<int> perm(count);
    SplitMix64 rng{seed};
    long t = 0;
    for (int e = 0; e < epochs; ++e) {
        for (int s = 0; s < count; ++s) perm[s] = s;
        for (int s = count - 1; s > 0; --s) {   // Fisher-Yates
            const int r = (int)(rng.next() % (uint64_t)(s + 1));
            const int tmp = perm[s];
            perm[s] = perm[r];
            perm[r] = tmp;
        }
        // the previous epoch's kernels read perm: wait before overwriting it
        HIP_TRY(hipStreamSynchronize(n->st));
        HIP_TRY(hipMemcpy(n->perm, perm.data(), sizeof(int) * (size_t)count, hipMemcpyHostToDevice));
        for (int b = 0; b < nbatch; ++b, ++t) {
            const int first = b * batch, cnt = count - first < batch ? count - first : batch;
            launch_mlp_grad(x_dev, y_dev, n->perm, first, cnt, n->view(), n->part, n->loss_part, nw, n->st);
            launch_mlp_reduce(n->part, nw, n->loss_part, n->grad, n->loss_acc, e, n->st);
            // cosine decay of the step size to 5 % over the run
            const double f = 0.05 + 0.95 * 0.5 * (1.0 + std::cos(M_PI * (double)t / (double)total));
            n->adam_t += 1;
            const float c1 = 1.0f - std::pow(b1, (float)n->adam_t), c2 = 1.0f - std::pow(b2, (float)n->adam_t);
            launch_mlp_adam(n->master, n->m1, n->m2, n->grad, (float)(lr * f), b1, b2, c1, c2, epsa, n->st);
            launch_mlp_pack(n->master, n->mut(), n->st);
        }
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(n->st));
    if (epoch_loss) {
        std::vector<float> l(epochs);
        HIP_TRY(hipMemcpy(l.data(), n->loss_acc, sizeof(float) * epochs, hipMemcpyDeviceToHost));
        for (int e = 0; e < epochs; ++e) epoch_loss[e] = l[e] / nbatch;
    }
    return MM_OK;
}

} // extern "C"
