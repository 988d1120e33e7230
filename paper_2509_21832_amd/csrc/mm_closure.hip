// mm_closure.hip -- kernels of the learned-closure form of the 2D2V step.
//
// The macro system of Sec. 5.1 is closed by the heat-flux tensor H of the micro
// part (eq5-41).  In near-continuum cells the closure form replaces the micro
// solve by a small network that predicts, from the local macro state and its
// first and second differences and its local mean free path, the heat-flux
// vector q, the stress deviation S and the
// traceless third moments t = (H111 - 3 H122, 3 H112 - H222) of eps g (scaled
// by 1/eps).  H is rebuilt from its contraction q (the heat-flux vector h of
// Sec. 6.3) and t: the isotropic form H_abc = (q_a d_bc + q_b d_ac + q_c d_ab) / 2
// plus t's traceless part.  Cells next to a non-periodic side, and cells
// whose local Knudsen indicator exceeds the threshold, keep the full micro
// solve; their neighbours' micro parts are rebuilt from (q, S, t) when needed.
//
// The network: 30 -> 64 -> 64 -> 7, exact (erf) GELU, bf16 weights and
// activations on the matrix cores (v_mfma_f32_32x32x16_bf16) with FP32
// accumulation, FP32 master weights and Adam moments.  Every matrix product of
// the forward and backward passes runs on a 32-sample tile per wavefront, with
// operands staged in LDS in plain row-major layouts.
#include <cstdint>

#include "mm_closure.h"
#include "mm_fused_common.h"

namespace mm {
namespace closure {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc (32 x 32) += A (32 x 16) B (16 x 32) with A(i, k) = a[i * ai + k * ak] and
// B(k, j) = b[k * bk + j * bj] (bf16 in LDS).  Operand layout of the gfx950
// instruction: lane r + 32 g holds A(r, 8 g + t) and B(8 g + t, r), t = 0..7.
__device__ __forceinline__ void mma(f32x16 &acc, const __bf16 *a, int ai, int ak, const __bf16 *b, int bk, int bj,
                                    int lane)
{
    const int r = lane & 31, g = lane >> 5;
    bf16x8 av, bv;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        av[t] = a[r * ai + (8 * g + t) * ak];
        bv[t] = b[(8 * g + t) * bk + r * bj];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
}

// accumulator slot v of a lane holds element (acc_row(v, lane), lane & 31)
__device__ __forceinline__ int acc_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

__device__ __forceinline__ f32x16 zero16()
{
    f32x16 z;
#pragma unroll
    for (int v = 0; v < 16; ++v) z[v] = 0.0f;
    return z;
}

// GELU without branches.  With a = |z|, erfc(a / sqrt 2) = 2^(-a Q(a)), Q the degree-5
// least-squares Chebyshev fit of -log2(erfc(a / sqrt 2)) / a on [0, 4 sqrt 2]
// (fit_erf.py; held at 4 sqrt 2 beyond, where erfc is below 2e-8).  For either sign,
//   z Phi(z) = max(z, 0) - a 2^(-a Q(a) - 1),
// within 2e-6 of the exact GELU, far below the bf16 rounding of the activations; the
// library erff takes a divergent branch at |x| = 1 and costs several times as much.
__device__ __forceinline__ float half_erfc(float a)     // erfc(a / sqrt 2) / 2, a >= 0
{
    constexpr float c[6] = {1.151109576e+00f, 4.590861499e-01f, 5.302880332e-02f, -7.888867520e-03f,
                            7.298647542e-04f, -3.054398985e-05f};
    const float ac = fminf(a, 5.65685424949238f);
    float q = c[5];
#pragma unroll
    for (int k = 4; k >= 0; --k) q = fmaf(q, ac, c[k]);
    return __builtin_amdgcn_exp2f(-fmaf(a, q, 1.0f));
}

__device__ __forceinline__ float gelu(float z)
{
    const float a = fabsf(z);
    return fmaf(-a, half_erfc(a), fmaxf(z, 0.0f));
}

__device__ __forceinline__ float gelu_d(float z)
{
    const float he = half_erfc(fabsf(z));
    const float Phi = z >= 0.0f ? 1.0f - he : he;
    return Phi + z * __builtin_amdgcn_exp2f(-0.72134752044448170f * z * z) * 0.39894228040143268f;
}

// Weights of the network in LDS (bf16): W1 [64][32] (inputs 30, 31 zero),
// W2 [64][64], W3 [32][64] (rows 7..31 zero); biases and normalisation FP32.
struct SmemW {
    __bf16 W1[NH * 32];
    __bf16 W2[NH * NH];
    __bf16 W3[32 * NH];
    float b1[NH], b2[NH], b3[16];
    float nrm[NNORM];
};

__device__ void load_weights(SmemW &s, const MlpDev &w)
{
    for (int t = threadIdx.x; t < NH * 32; t += blockDim.x) s.W1[t] = w.W1[t];
    for (int t = threadIdx.x; t < NH * NH; t += blockDim.x) s.W2[t] = w.W2[t];
    for (int t = threadIdx.x; t < 32 * NH; t += blockDim.x) s.W3[t] = w.W3[t];
    for (int t = threadIdx.x; t < NH; t += blockDim.x) {
        s.b1[t] = w.b1[t];
        s.b2[t] = w.b2[t];
    }
    for (int t = threadIdx.x; t < 16; t += blockDim.x) s.b3[t] = t < NO ? w.b3[t] : 0.0f;
    for (int t = threadIdx.x; t < NNORM; t += blockDim.x) s.nrm[t] = w.norm[t];
    __syncthreads();
}

// Per-wavefront activations of one 32-sample tile (row-major, column = sample)
struct SmemFwd {
    __bf16 X[32 * 32];     // normalised inputs [feature][sample], features >= 30 zero
    __bf16 A1[NH * 32];
    __bf16 A2[NH * 32];
};

struct SmemBwd {
    float G1[NH * 32];     // gelu'(z1), gelu'(z2)
    float G2[NH * 32];
    __bf16 dY[32 * 32];    // output error [output][sample], outputs >= 7 zero
    __bf16 dZ2[NH * 32];
    __bf16 dZ1[NH * 32];
};

// Forward pass of one tile: samples s0 .. s0+31 (rows idx[s] of X when idx is
// given), normalised outputs yh[o] of sample (lane & 31) for o = 4 (lane >> 5) + v,
// v < 4 (o < 7 only).  With bw, gelu'(z) is kept for the backward pass.
template <bool TRAIN>
__device__ void forward_tile(const SmemW &W, SmemFwd &F, SmemBwd *Bw, const float *__restrict__ X,
                             const int *__restrict__ idx, int s0, int n, int lane, float (&yh)[4])
{
    // normalised inputs
    for (int t = lane; t < 32 * 32; t += 64) {
        const int f = t >> 5, j = t & 31;
        const int s = s0 + j;
        float x = 0.0f;
        if (f < NF && s < n) {
            const int row = idx ? idx[s] : s;
            x = (X[(size_t)row * NF + f] - W.nrm[f]) / W.nrm[NF + f];
        }
        F.X[t] = (__bf16)x;
    }
    wave_sync();
    const int j = lane & 31;
    // layer 1: Z1^T (64 x 32) = W1 (64 x 32) X (32 x 32)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = zero16();
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            mma(acc, W.W1 + 32 * mt * 32 + 16 * kb, 32, 1, F.X + 16 * kb * 32, 32, 1, lane);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 32 * mt + acc_row(v, lane);
            const float z = acc[v] + W.b1[h];
            F.A1[h * 32 + j] = (__bf16)gelu(z);
            if constexpr (TRAIN) Bw->G1[h * 32 + j] = gelu_d(z);
        }
    }
    wave_sync();
    // layer 2: Z2^T = W2 (64 x 64) A1 (64 x 32)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = zero16();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            mma(acc, W.W2 + 32 * mt * NH + 16 * kb, NH, 1, F.A1 + 16 * kb * 32, 32, 1, lane);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 32 * mt + acc_row(v, lane);
            const float z = acc[v] + W.b2[h];
            F.A2[h * 32 + j] = (__bf16)gelu(z);
            if constexpr (TRAIN) Bw->G2[h * 32 + j] = gelu_d(z);
        }
    }
    wave_sync();
    // layer 3: Yh^T (rows 0..6 of 32) = W3 (32 x 64, rows >= 7 zero) A2
    f32x16 acc = zero16();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) mma(acc, W.W3 + 16 * kb, NH, 1, F.A2 + 16 * kb * 32, 32, 1, lane);
    // slots v < 4 hold rows o = 4 (lane >> 5) + v (rows 0..7); rows 8.. are unused
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = acc_row(v, lane);
        yh[v] = o < NO ? acc[v] + W.b3[o] : 0.0f;
    }
}

// ------------------------------------------------------------- inference

// The network's weights in VGPRs, in the per-lane operand order (Wp)
struct MlpRegs {
    bf16x8 w1[4], w2[8], w3[4];
};

__device__ __forceinline__ void mlp_regs(const __bf16 *__restrict__ Wp, int lane, MlpRegs &R)
{
    const bf16x8 *p = (const bf16x8 *)Wp;
#pragma unroll
    for (int b = 0; b < 4; ++b) R.w1[b] = p[b * 64 + lane];
#pragma unroll
    for (int b = 0; b < 8; ++b) R.w2[b] = p[(4 + b) * 64 + lane];
#pragma unroll
    for (int b = 0; b < 4; ++b) R.w3[b] = p[(12 + b) * 64 + lane];
}

// Forward pass of the 32 samples of a wavefront with no LDS traffic: lane
// (r, g) holds sample r's normalised inputs x; every layer's accumulator slots
// are the next layer's B operand (the packed weights carry the matching
// column order).  Returns the normalised outputs o = 4 g + v (v < 4, o < 7).
__device__ __forceinline__ void mlp_eval(const MlpRegs &R, const float *b1, const float *b2, const float *b3,
                                         const float (&x)[NF], int lane, float (&yh)[4])
{
    const int g = lane >> 5;
    bf16x8 B1[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int f0 = 16 * kb + q, f1 = 16 * kb + 8 + q;
            const float v0 = f0 < NF ? x[f0 < NF ? f0 : 0] : 0.0f, v1 = f1 < NF ? x[f1 < NF ? f1 : 0] : 0.0f;
            B1[kb][q] = (__bf16)(g ? v1 : v0);
        }
    bf16x8 B2[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = zero16();
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.w1[2 * mt + kb], B1[kb], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 16; ++v)
            B2[2 * mt + (v >> 3)][v & 7] = (__bf16)gelu(acc[v] + b1[32 * mt + acc_row(v, lane)]);
    }
    bf16x8 B3[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = zero16();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.w2[4 * mt + kb], B2[kb], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 16; ++v)
            B3[2 * mt + (v >> 3)][v & 7] = (__bf16)gelu(acc[v] + b2[32 * mt + acc_row(v, lane)]);
    }
    f32x16 acc = zero16();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.w3[kb], B3[kb], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = 4 * g + v;
        yh[v] = o < NO ? acc[v] + b3[o < NO ? o : 0] : 0.0f;
    }
}

// Y = MLP(X) (accumulate = 0) or Y += scale MLP(X) (accumulate = 1)
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ X, int n, MlpDev w,
                                                     float *__restrict__ Y, int accumulate, float scale)
{
    __shared__ float sb[NH + NH + 16 + NNORM + NF];
    for (int t = threadIdx.x; t < NH; t += blockDim.x) {
        sb[t] = w.b1[t];
        sb[NH + t] = w.b2[t];
    }
    for (int t = threadIdx.x; t < 16; t += blockDim.x) sb[2 * NH + t] = t < NO ? w.b3[t] : 0.0f;
    for (int t = threadIdx.x; t < NNORM; t += blockDim.x) sb[2 * NH + 16 + t] = w.norm[t];
    // reciprocals of the input scales, once per workgroup (the inputs are then multiplied)
    for (int t = threadIdx.x; t < NF; t += blockDim.x) sb[2 * NH + 16 + NNORM + t] = 1.0f / w.norm[NF + t];
    __syncthreads();
    const float *b1 = sb, *b2 = sb + NH, *b3 = sb + 2 * NH, *nrm = sb + 2 * NH + 16, *isd = nrm + NNORM;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    MlpRegs R;
    mlp_regs(w.Wp, lane, R);
    const int ntile = (n + 31) / 32;
    for (int tile = blockIdx.x * 4 + wv; tile < ntile; tile += gridDim.x * 4) {
        const int s = tile * 32 + (lane & 31);
        float x[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) x[f] = s < n ? (X[(size_t)s * NF + f] - nrm[f]) * isd[f] : 0.0f;
        float yh[4];
        mlp_eval(R, b1, b2, b3, x, lane, yh);
        if (s < n) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 4 * (lane >> 5) + v;
                if (o < NO) {
                    const float y = yh[v] * nrm[2 * NF + NO + o] + nrm[2 * NF + o];
                    Y[(size_t)s * NO + o] = accumulate ? Y[(size_t)s * NO + o] + scale * y : y;
                }
            }
        }
    }
}

// ------------------------------------------------------------- training

// Gradient of the normalised mean-square loss over `count` samples idx[first ..
// first + count) (mean over samples and outputs: scale = 1 / (7 count)).  Each
// wavefront works on tiles tile0 + w, tile0 + w + nw, ... and writes its
// partial gradient (parameter layout of the oracle) and loss to part[wave].
__global__ __launch_bounds__(128) void k_mlp_grad(const float *__restrict__ X, const float *__restrict__ Yt,
                                                  const int *__restrict__ idx, int first, int count, MlpDev w,
                                                  float *__restrict__ part, float *__restrict__ loss_part)
{
    __shared__ SmemW W;
    __shared__ SmemFwd F[2];
    __shared__ SmemBwd Bw[2];
    load_weights(W, w);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * 2 + wv, nw = gridDim.x * 2;
    const int j = lane & 31;
    const float scale = 1.0f / (float)(NO * count);
    const int ntile = (count + 31) / 32;
    SmemFwd &Fw = F[wv];
    SmemBwd &B = Bw[wv];
    f32x16 gW1[2], gW2[4], gW3[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) gW1[q] = gW3[q] = zero16();
#pragma unroll
    for (int q = 0; q < 4; ++q) gW2[q] = zero16();
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, loss = 0.f;   // lane l: bias sums of unit l (outputs: l < 7)
    const float *Xt = idx ? X : X + (size_t)first * NF;   // tile rows: idx[first + s], or first + s

    for (int tile = gw; tile < ntile; tile += nw) {
        const int s0 = tile * 32;
        float yh[4];
        forward_tile<true>(W, Fw, &B, Xt, idx ? idx + first : nullptr, s0, count, lane, yh);
        // output error dY (bf16), rows >= 7 zero
        for (int t = lane; t < 32 * 32; t += 64) B.dY[t] = (__bf16)0.0f;
        wave_sync();
        {
            const int s = s0 + j;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 4 * (lane >> 5) + v;
                if (o < NO && s < count) {
                    const int row = idx ? idx[first + s] : first + s;
                    const float t = (Yt[(size_t)row * NO + o] - W.nrm[2 * NF + o]) / W.nrm[2 * NF + NO + o];
                    const float r = yh[v] - t;
                    loss += r * r;
                    B.dY[o * 32 + j] = (__bf16)(2.0f * r * scale);
                }
            }
        }
        wave_sync();
        // dW3 (32 x 64: rows o) += dY (32 x 32, [o][s]) A2^T (32 x 64: A2[h][s])
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                mma(gW3[nt], B.dY + 16 * kb, 32, 1, Fw.A2 + 32 * nt * 32 + 16 * kb, 1, 32, lane);
        // dA2^T (64 x 32) = W3^T (64 x 16) dY (16 x 32); dZ2 = dA2 gelu'(z2)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            f32x16 acc = zero16();
            mma(acc, W.W3 + 32 * mt, 1, NH, B.dY, 32, 1, lane);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int h = 32 * mt + acc_row(v, lane);
                B.dZ2[h * 32 + j] = (__bf16)(acc[v] * B.G2[h * 32 + j]);
            }
        }
        wave_sync();
        // dW2 (64 x 64) += dZ2 (64 x 32) A1^T (32 x 64)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int kb = 0; kb < 2; ++kb)
                    mma(gW2[mt * 2 + nt], B.dZ2 + 32 * mt * 32 + 16 * kb, 32, 1, Fw.A1 + 32 * nt * 32 + 16 * kb, 1,
                        32, lane);
        // dA1^T (64 x 32) = W2^T (64 x 64) dZ2 (64 x 32); dZ1 = dA1 gelu'(z1)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            f32x16 acc = zero16();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) mma(acc, W.W2 + 16 * kb * NH + 32 * mt, 1, NH, B.dZ2 + 16 * kb * 32, 32, 1, lane);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int h = 32 * mt + acc_row(v, lane);
                B.dZ1[h * 32 + j] = (__bf16)(acc[v] * B.G1[h * 32 + j]);
            }
        }
        wave_sync();
        // dW1 (64 x 32) += dZ1 (64 x 32) X^T (32 x 32)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                mma(gW1[mt], B.dZ1 + 32 * mt * 32 + 16 * kb, 32, 1, Fw.X + 16 * kb, 1, 32, lane);
        // bias gradients: sums over the tile's samples of the (bf16) errors;
        // lane l owns hidden unit l and, for l < 7, output l
        for (int jj = 0; jj < 32; ++jj) {
            gb1 += (float)B.dZ1[lane * 32 + jj];
            gb2 += (float)B.dZ2[lane * 32 + jj];
            if (lane < NO) gb3 += (float)B.dY[lane * 32 + jj];
        }
        wave_sync();
    }
    // partial gradient of this wavefront in the parameter layout
    float *g = part + (size_t)gw * NPARAM;
    float *gw1 = g, *gb1p = gw1 + NH * NF, *gw2 = gb1p + NH, *gb2p = gw2 + NH * NH, *gw3 = gb2p + NH,
          *gb3p = gw3 + NO * NH;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 32 * mt + acc_row(v, lane), f = j;
            if (f < NF) gw1[h * NF + f] = gW1[mt][v];
        }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 32 * (q >> 1) + acc_row(v, lane), k = 32 * (q & 1) + j;
            gw2[h * NH + k] = gW2[q][v];
        }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = acc_row(v, lane), h = 32 * nt + j;
            if (o < NO) gw3[o * NH + h] = gW3[nt][v];
        }
    gb1p[lane] = gb1;
    gb2p[lane] = gb2;
    if (lane < NO) gb3p[lane] = gb3;
    // loss: lanes hold disjoint terms; reduce over the wavefront
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (lane == 0) loss_part[gw] = loss * scale;
}

// sum of the partial gradients in a fixed order
__global__ void k_mlp_reduce(const float *__restrict__ part, int nparts, const float *__restrict__ loss_part,
                             float *__restrict__ grad, float *__restrict__ loss_acc, int loss_slot)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) {
        float s = 0.0f;
        for (int w = 0; w < nparts; ++w) s += part[(size_t)w * NPARAM + p];
        grad[p] = s;
    }
    if (p == 0 && loss_acc) {
        float s = 0.0f;
        for (int w = 0; w < nparts; ++w) s += loss_part[w];
        loss_acc[loss_slot] += s;
    }
}

// Adam step on the FP32 master weights, then the bf16 copies in matrix-core layout
__global__ void k_mlp_adam(float *__restrict__ master, float *__restrict__ m1, float *__restrict__ m2,
                           const float *__restrict__ grad, float lr, float b1, float b2, float c1, float c2,
                           float epsa)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.0f - b1) * g;
    const float b = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = b;
    master[p] -= lr * (a / c1) / (sqrtf(b / c2) + epsa);
}

// hidden unit carried by K index 8 g + t of K-block kb when the next layer's B
// operand is taken straight from this layer's accumulator slots: the slot
// v = 8 (kb % 2) + t of tile kb / 2 in lane group g holds row 8 (v / 4) + 4 g + v % 4
__device__ __forceinline__ int hidden_of(int kb, int g, int t)
{
    return 32 * (kb >> 1) + 16 * (kb & 1) + 8 * (t >> 2) + 4 * g + (t & 3);
}

__global__ void k_mlp_pack(const float *__restrict__ master, __bf16 *__restrict__ W1, __bf16 *__restrict__ W2,
                           __bf16 *__restrict__ W3, __bf16 *__restrict__ Wp, float *__restrict__ b1,
                           float *__restrict__ b2, float *__restrict__ b3)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const float *w1 = master, *pb1 = w1 + NH * NF, *w2 = pb1 + NH, *pb2 = w2 + NH * NH, *w3 = pb2 + NH,
                *pb3 = w3 + NO * NH;
    if (t < NWP) {
        // per-lane operand order: block b, lane (r, g), slot q
        const int b = t >> 9, lane = (t >> 3) & 63, q = t & 7, r = lane & 31, g = lane >> 5;
        float v;
        if (b < 4) {             // layer 1: tile mt, K-block kb (inputs in natural order)
            const int mt = b >> 1, kb = b & 1, f = 16 * kb + 8 * g + q;
            v = f < NF ? w1[(32 * mt + r) * NF + f] : 0.0f;
        } else if (b < 12) {     // layer 2: tile mt, K-block kb (inputs in accumulator order)
            const int mt = (b - 4) >> 2, kb = (b - 4) & 3;
            v = w2[(32 * mt + r) * NH + hidden_of(kb, g, q)];
        } else {                 // layer 3: K-block kb
            const int kb = b - 12;
            v = r < NO ? w3[r * NH + hidden_of(kb, g, q)] : 0.0f;
        }
        Wp[t] = (__bf16)v;
    }
    if (t < NH * 32) {
        const int h = t / 32, f = t % 32;
        W1[t] = (__bf16)(f < NF ? w1[h * NF + f] : 0.0f);
    }
    if (t < NH * NH) W2[t] = (__bf16)w2[t];
    if (t < 32 * NH) {
        const int o = t / NH, h = t % NH;
        W3[t] = (__bf16)(o < NO ? w3[o * NH + h] : 0.0f);
    }
    if (t < NH) {
        b1[t] = pb1[t];
        b2[t] = pb2[t];
    }
    if (t < NO) b3[t] = pb3[t];
}

// Mean and standard deviation of the 30 feature and 7 target columns (FP64
// sums, one workgroup per column).  A standard deviation below 1e-6 times the
// column's root mean square (or exactly zero) is raised to that floor.
__global__ __launch_bounds__(256) void k_mlp_norm(const float *__restrict__ X, const float *__restrict__ Y, int n,
                                                  float *__restrict__ norm)
{
    __shared__ double lds[4 * 2];
    const int col = blockIdx.x;
    const bool isx = col < NF;
    const float *A = isx ? X : Y;
    const int ld = isx ? NF : NO, c = isx ? col : col - NF;
    double v[2] = {0.0, 0.0};
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const double a = A[(size_t)s * ld + c];
        v[0] += a;
        v[1] += a * a;
    }
    block_sum<2, 4>(v, lds);
    if (threadIdx.x == 0) {
        const double mean = v[0] / n, ms = v[1] / n;
        double var = ms - mean * mean;
        if (var < 0.0) var = 0.0;
        double sd = sqrt(var);
        const double floor = 1e-6 * sqrt(ms) + 1e-30;
        if (sd < floor) sd = floor;
        if (isx) {
            norm[c] = (float)mean;
            norm[NF + c] = (float)sd;
        } else {
            norm[2 * NF + c] = (float)mean;
            norm[2 * NF + NO + c] = (float)sd;
        }
    }
}

// ------------------------------------------------------------- the solver side

__device__ __forceinline__ void prim(const double *q, double *w)
{
    const double rho = q[0], ir = 1.0 / rho, u1 = q[1] * ir, u2 = q[2] * ir;
    const double P11 = q[3] - rho * u1 * u1, P12 = q[4] - rho * u1 * u2, P22 = q[5] - rho * u2 * u2;
    w[0] = rho; w[1] = u1; w[2] = u2; w[3] = 0.5 * (P11 + P22) * ir;
    w[4] = P11; w[5] = P12; w[6] = P22;
}

// features of cell c rounded to FP32 (as stored for training), local Knudsen
// indicator (FP64 from the FP64 features) and the next-to-a-non-periodic-side flag
__device__ __forceinline__ void cell_features(const double *__restrict__ Q, const Params &P, int c, float (&fo)[NF],
                                              double &kn, bool &edge)
{
    const int i = c % P.nx, j = c / P.nx;
    const bool px = P.bc[0].kind == BC_PERIODIC, py = P.bc[2].kind == BC_PERIODIC;
    int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
    bool hm = true, hp = true, vm = true, vp = true;
    if (im < 0) { if (px) im = P.nx - 1; else { hm = false; im = i; } }
    if (ip >= P.nx) { if (px) ip = 0; else { hp = false; ip = i; } }
    if (jm < 0) { if (py) jm = P.ny - 1; else { vm = false; jm = j; } }
    if (jp >= P.ny) { if (py) jp = 0; else { vp = false; jp = j; } }
    double w0[7], wxm[7], wxp[7], wym[7], wyp[7];
    prim(Q + 6 * (size_t)c, w0);
    prim(Q + 6 * (size_t)(j * P.nx + im), wxm);
    prim(Q + 6 * (size_t)(j * P.nx + ip), wxp);
    prim(Q + 6 * (size_t)(jm * P.nx + i), wym);
    prim(Q + 6 * (size_t)(jp * P.nx + i), wyp);
    double f[NF];
    // A missing neighbour was loaded from the cell itself (wxp = w0 when !hp, ...),
    // so wxp - wxm is the centred difference times 2 dx, the one-sided one times dx,
    // or zero: one scale per direction picks the divisor.
    const double idx = 1.0 / P.dx, idy = 1.0 / P.dy;
    const double sx = (hm && hp) ? 0.5 * idx : idx, sy = (vm && vp) ? 0.5 * idy : idy;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        f[a] = w0[a];
        f[7 + a] = (wxp[a] - wxm[a]) * sx;
        f[14 + a] = (wyp[a] - wym[a]) * sy;
    }
    // the local mean free path eps sqrt(T) / tau, and the second differences of
    // (rho, u1, u2, T) along x and y (zero next to a side that is not periodic:
    // those cells are always solved)
    const double rho = w0[0], T = w0[3];
    const double lam = P.eps * sqrt(T) / tau_of(P, rho, rho * T, T);
    f[21] = lam;
    const double sxx = (hm && hp) ? idx * idx : 0.0, syy = (vm && vp) ? idy * idy : 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        f[22 + a] = (wxp[a] - 2.0 * w0[a] + wxm[a]) * sxx;
        f[26 + a] = (wyp[a] - 2.0 * w0[a] + wym[a]) * syy;
    }
#pragma unroll
    for (int a = 0; a < NF; ++a) fo[a] = (float)f[a];
    const double gr = sqrt(f[7] * f[7] + f[14] * f[14]) / rho;
    const double gT = sqrt(f[10] * f[10] + f[17] * f[17]) / T;
    const double gu = sqrt(f[8] * f[8] + f[15] * f[15] + f[9] * f[9] + f[16] * f[16]) / sqrt(T);
    const double m = fmax(gr, fmax(gT, gu));
    kn = lam * m;
    edge = (!px && (i == 0 || i == P.nx - 1)) || (!py && (j == 0 || j == P.ny - 1));
}

// features (FP32), local Knudsen indicator and the always-micro mask per cell
__global__ void k_features2d(const double *__restrict__ Q, Params P, float *__restrict__ feat,
                             float *__restrict__ kn, uint8_t *__restrict__ edge)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.nx * P.ny) return;
    float f[NF];
    double k;
    bool e;
    cell_features(Q, P, c, f, k, e);
#pragma unroll
    for (int a = 0; a < NF; ++a) feat[(size_t)c * NF + a] = f[a];
    kn[c] = (float)k;
    edge[c] = e;
}

// Navier-Stokes-Fourier values of (q, S, t) / eps from the features of a cell:
// q = -(2 p / tau) grad T, S = -(p / tau) sigma + nu (P - p I) / eps and t = 0,
// the moments of the first-order micro part G-hat (eqn5-97) with the ES term
__device__ __forceinline__ void nsf_out(const float *f, const Params &P, double o[NO])
{
    const double rho = f[0], T = f[3], p = rho * T, tau = tau_of(P, rho, p, T);
    const double s11 = (double)f[8] - f[16], s12 = (double)f[15] + f[9];
    o[0] = -2.0 * p / tau * f[10];
    o[1] = -2.0 * p / tau * f[17];
    o[2] = -(p / tau) * s11 + P.nu * (f[4] - p) / P.eps;
    o[3] = -(p / tau) * s12 + P.nu * f[5] / P.eps;
    o[4] = (p / tau) * s11 + P.nu * (f[6] - p) / P.eps;
    o[5] = 0.0;
    o[6] = 0.0;
}

// H (H111, H112, H122, H222) of a closure cell from q and the traceless part
// t = (H111 - 3 H122, 3 H112 - H222): the isotropic form of q plus t's part
__device__ __forceinline__ void closure_H(double q1, double q2, double t1, double t2, double *H)
{
    H[0] = 1.5 * q1 + 0.25 * t1;
    H[1] = 0.5 * q2 + 0.25 * t2;
    H[2] = 0.5 * q1 - 0.25 * t1;
    H[3] = 1.5 * q2 - 0.25 * t2;
}

__global__ void k_nsf2d(const float *__restrict__ feat, int n, Params P, float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double o[NO];
    nsf_out(feat + (size_t)c * NF, P, o);
#pragma unroll
    for (int k = 0; k < NO; ++k) out[(size_t)c * NO + k] = (float)o[k];
}

// Cell classes: micro (1) next to a non-periodic side or where kn > kn_max,
// closure (0) elsewhere; closure cells get H of eps (q, t).
__global__ void k_classify2d(const float *__restrict__ kn, const uint8_t *__restrict__ edge,
                             const float *__restrict__ out, int n, float kn_max, double eps,
                             uint8_t *__restrict__ cls, double *__restrict__ H,
                             unsigned long long *__restrict__ nclosure, int *__restrict__ nrebuild)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) *nrebuild = 0;       // the list of k_need2d starts empty
    bool closure = false;
    if (c < n) {
        const bool micro = edge[c] || !(kn[c] <= kn_max);
        cls[c] = micro ? 1 : 0;
        closure = !micro;
        if (closure) {
            const float *o = out + (size_t)c * NO;
            closure_H(eps * o[0], eps * o[1], eps * o[5], eps * o[6], H + 4 * (size_t)c);
        }
    }
    // count of closure cells: per-wavefront ballots, one atomic per workgroup
    __shared__ int wcount[4];
    const unsigned long long b = __ballot(closure);
    if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = (int)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (tot) atomicAdd(nclosure, (unsigned long long)tot);
    }
}

// The closure part of a step for 32 cells per wavefront: features and
// indicator (both lane halves of a cell compute them), classes, the closure
// values out = (q, S, t) / eps (NSF; the network; or NSF plus scale x network)
// and H of the closure cells.  Lane half g holds outputs o = 4 g + v.
template <bool NET>
__global__ __launch_bounds__(256) void k_cells2d(const double *__restrict__ Q, Params P, MlpDev w, int residual,
                                                 float kn_max, uint8_t *__restrict__ cls, float *__restrict__ out,
                                                 double *__restrict__ H, unsigned long long *__restrict__ nclosure,
                                                 int *__restrict__ nrebuild)
{
    __shared__ float sb[NH + NH + 16 + NNORM + NF];
    __shared__ int wcount[4];
    if (blockIdx.x == 0 && threadIdx.x == 0) *nrebuild = 0;     // the list of k_need2d starts empty
    const int n = P.nx * P.ny;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 5;
    if constexpr (NET) {
        for (int t = threadIdx.x; t < NH; t += blockDim.x) {
            sb[t] = w.b1[t];
            sb[NH + t] = w.b2[t];
        }
        for (int t = threadIdx.x; t < 16; t += blockDim.x) sb[2 * NH + t] = t < NO ? w.b3[t] : 0.0f;
        for (int t = threadIdx.x; t < NNORM; t += blockDim.x) sb[2 * NH + 16 + t] = w.norm[t];
        for (int t = threadIdx.x; t < NF; t += blockDim.x) sb[2 * NH + 16 + NNORM + t] = 1.0f / w.norm[NF + t];
        __syncthreads();
    }
    const float *b1 = sb, *b2 = sb + NH, *b3 = sb + 2 * NH, *nrm = sb + 2 * NH + 16, *isd = nrm + NNORM;
    const int c = (blockIdx.x * 4 + wv) * 32 + (lane & 31);
    const bool valid = c < n;
    float f[NF];
    double kn = 0.0;
    bool edge = true;
    if (valid) cell_features(Q, P, c, f, kn, edge);
    else
        for (int a = 0; a < NF; ++a) f[a] = 1.0f;
    const bool micro = edge || !((float)kn <= kn_max);     // the decision in FP32, as for stored indicators
    // closure values of this lane's outputs o = 4 g + v
    double o4[4] = {0.0, 0.0, 0.0, 0.0};
    if (!NET || residual) {
        double b[NO];
        nsf_out(f, P, b);
        // outputs 4 g + v: a select per slot, not an index that depends on the lane
#pragma unroll
        for (int v = 0; v < 4; ++v) o4[v] = g ? (4 + v < NO ? b[4 + v < NO ? 4 + v : 0] : 0.0) : b[v];
    }
    if constexpr (NET) {
        MlpRegs R;
        mlp_regs(w.Wp, lane, R);
        float x[NF];
#pragma unroll
        for (int a = 0; a < NF; ++a) x[a] = (f[a] - nrm[a]) * isd[a];
        float yh[4];
        mlp_eval(R, b1, b2, b3, x, lane, yh);
        const float scale = residual == 2 ? (float)P.eps : 1.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 4 * g + v;
            if (o < NO) {
                const float y = yh[v] * nrm[2 * NF + NO + o] + nrm[2 * NF + o];
                // the same FP32 arithmetic as the separate forward kernel
                o4[v] = residual ? (double)((float)o4[v] + scale * y) : (double)y;
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) o4[v] = (double)(float)o4[v];
    }
    // t = outputs 5, 6: slots 1, 2 of the other lane half
    const double t1 = __shfl_xor(o4[1], 32, 64), t2 = __shfl_xor(o4[2], 32, 64);
    if (valid) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 4 * g + v;
            if (o < NO) out[(size_t)c * NO + o] = (float)o4[v];
        }
        if (g == 0) {
            cls[c] = micro ? 1 : 0;
            if (!micro)
                closure_H(P.eps * (double)(float)o4[0], P.eps * (double)(float)o4[1], P.eps * (double)(float)t1,
                          P.eps * (double)(float)t2, H + 4 * (size_t)c);
        }
    }
    // closure cells of the workgroup (lane half 0 of each wavefront), one atomic
    const unsigned long long bal = __ballot(valid && g == 0 && !micro);
    if (lane == 0) wcount[wv] = (int)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (tot) atomicAdd(nclosure, (unsigned long long)tot);
    }
}

// Cells whose micro part a solved cell needs (its 3 x 3 block) but whose G^n is
// not current go to a list; the validity of G^{n+1} (= solved) goes to
// valid_next.  One thread per cell, NEED_BLOCK cells per workgroup and one list
// atomic per workgroup: the cells next to the walls all need rebuilding, and an
// atomic per wavefront on the one counter serialised about 500 of them.
constexpr int NEED_BLOCK = 1024;

__global__ __launch_bounds__(NEED_BLOCK) void k_need2d(const uint8_t *__restrict__ cls, const uint8_t *__restrict__ valid,
                         uint8_t *__restrict__ valid_next, int *__restrict__ list, int *__restrict__ nrebuild,
                         Params P)
{
    __shared__ int wcount[NEED_BLOCK / 64], wbase[NEED_BLOCK / 64];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in_grid = c < P.nx * P.ny;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cc = in_grid ? c : 0;
    const int i = cc % P.nx, j = cc / P.nx;
    const bool px = P.bc[0].kind == BC_PERIODIC, py = P.bc[2].kind == BC_PERIODIC;
    bool need = false;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
            int ii = i + di, jj = j + dj;
            bool in = true;
            if (ii < 0 || ii >= P.nx) {
                in = px;
                ii = ii < 0 ? ii + P.nx : ii - P.nx;
            }
            if (jj < 0 || jj >= P.ny) {
                in = in && py;
                jj = jj < 0 ? jj + P.ny : jj - P.ny;
            }
            if (in && cls[jj * P.nx + ii]) need = true;
        }
    if (in_grid) valid_next[c] = cls[c];
    // the workgroup's listed cells: wavefront counts, one atomic reserves the
    // workgroup's slots, each lane takes its wavefront's offset plus its rank
    const bool add = in_grid && need && !valid[c];
    const uint64_t m = __ballot(add);
    if (lane == 0) wcount[wv] = (int)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < NEED_BLOCK / 64; ++w) {
            wbase[w] = tot;
            tot += wcount[w];
        }
        const int base = tot ? atomicAdd(nrebuild, tot) : 0;
        for (int w = 0; w < NEED_BLOCK / 64; ++w) wbase[w] += base;
    }
    __syncthreads();
    if (add) list[wbase[wv] + __popcll(m & ((1ull << lane) - 1))] = c;
}

// Rebuild the listed cells from their (q, S, t) / eps:
//   g = M / (2 p T) [S' : w w^T + (q . w)(|w|^2 / (2T) - 2)]
//       + M / (24 p T^2) [t1 (w1^3 - 3 w1 w2^2) + t2 (3 w1^2 w2 - w2^3)],
// then (I - Pi) g, with S' the traceless part of S (the cubic harmonics have
// zero moments below third order and third moments t, as 24 rho T^3 / (24 p T^2) = 1).  A fixed grid of wavefronts walks the list,
// one cell per wavefront at a time.
template <typename TS>
__global__ __launch_bounds__(256) void k_rebuild2d(TS *__restrict__ G, const double *__restrict__ rec,
                                                   const float *__restrict__ out, const int *__restrict__ list,
                                                   const int *__restrict__ nrebuild, Params P)
{
    const int lane = threadIdx.x & 63;
    const int w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int nw = gridDim.x * 4;
    const int count = *nrebuild;
    for (int t = w0; t < count; t += nw) {
        const int c = __builtin_amdgcn_readfirstlane(list[t]);
        const double *R = rec + (size_t)c * REC;
        fused::Cell<double> cl;
        fused::load_cell(R, cl);
        const double T = R[R_T], rho = R[R_RHO], p = rho * T;
        const float *o = out + (size_t)c * NO;
        const double q1 = o[0], q2 = o[1];
        const double tr = 0.5 * ((double)o[2] + o[4]);
        const double a11 = o[2] - tr, a12 = o[3], a22 = o[4] - tr;
        const double pre = 1.0 / (2.0 * p * T), pre3 = pre / (12.0 * T);
        const double c1 = pre3 * o[5], c2 = pre3 * o[6];
        // t1 (w1^3 - 3 w1 w2^2) + t2 (3 w1^2 w2 - w2^3), scaled by pre3
        auto cubic = [&](double w1, double w2) {
            const double a = w1 * w1, b = w2 * w2;
            return c1 * w1 * (a - 3.0 * b) + c2 * w2 * (3.0 * a - b);
        };
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        if (lk_lanes(P.nv1, P.nv2) == 64) {
            // lane-k layout: lane (k, l0) owns the nodes (k, l0 + L m); the Maxwellian
            // follows e(m+1) = e(m) r(m), r(m+1) = r(m) kappa along them
            const int L = 64 / P.nv1, k = lane % P.nv1, l0 = lane / P.nv1, npt = P.nv / 64;
            const double i2T = R[R_I2T], h = L * P.dv2;
            const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2b = P.v2_lo + (l0 + 0.5) * P.dv2;
            const double w1 = v1 - cl.u1d, w2b = v2b - cl.u2d;
            const double e0 = R[R_MPRE] * exp(-(w1 * w1 + w2b * w2b) * i2T);
            const double r0 = exp(-(2.0 * w2b + h) * h * i2T), kap = R[R_KM];
            const double b0 = pre * a11 * w1 * w1, b1 = pre * 2.0 * a12 * w1, b2 = pre * a22, bq = pre * q1 * w1;
            auto gval = [&](double w2, double M) {
                const double ww = w1 * w1 + w2 * w2;
                return M * (b0 + (b1 + b2 * w2) * w2 + (bq + pre * q2 * w2) * (ww * i2T - 2.0) + cubic(w1, w2));
            };
            double e = e0, r = r0;
            for (int m = 0; m < npt; ++m) {
                const double v2 = v2b + m * h, g = gval(v2 - cl.u2d, e);
                e *= r;
                r *= kap;
                s[0] += g;
                s[1] += v1 * g;
                s[2] += v2 * g;
                s[3] += (v1 * v1 + v2 * v2) * g;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
#pragma unroll
                for (int a = 0; a < 4; ++a) s[a] += __shfl_xor(s[a], off, 64);
            double cp[4];
            fused::proj_poly(cl, s, cp);
            TS *gout = G + (size_t)c * P.nv;
            e = e0;
            r = r0;
            for (int m = 0; m < npt; ++m) {
                const double v2 = v2b + m * h, g = gval(v2 - cl.u2d, e);
                const double pg = (cp[0] + cp[1] * v1 + cp[2] * v2 + cp[3] * (v1 * v1 + v2 * v2)) * e;
                e *= r;
                r *= kap;
                gout[lane + 64 * m] = (TS)(g - pg);
            }
            continue;
        }
        // raw values and their (1, v1, v2, |v|^2) sums
        for (int n = lane; n < P.nv; n += 64) {
            const int k = n % P.nv1, l = n / P.nv1;
            const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
            const double w1 = v1 - cl.u1d, w2 = v2 - cl.u2d, ww = w1 * w1 + w2 * w2;
            const double M = R[R_MPRE] * exp(-ww * R[R_I2T]);
            const double g = M * (pre * (a11 * w1 * w1 + 2.0 * a12 * w1 * w2 + a22 * w2 * w2 +
                                         (q1 * w1 + q2 * w2) * (ww / (2.0 * T) - 2.0)) +
                                  cubic(w1, w2));
            s[0] += g;
            s[1] += v1 * g;
            s[2] += v2 * g;
            s[3] += (v1 * v1 + v2 * v2) * g;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int a = 0; a < 4; ++a) s[a] += __shfl_xor(s[a], off, 64);
        double cp[4];
        fused::proj_poly(cl, s, cp);
        TS *gout = G + (size_t)c * P.nv;
        for (int n = lane; n < P.nv; n += 64) {
            const int k = n % P.nv1, l = n / P.nv1;
            const double v1 = P.v1_lo + (k + 0.5) * P.dv1, v2 = P.v2_lo + (l + 0.5) * P.dv2;
            const double w1 = v1 - cl.u1d, w2 = v2 - cl.u2d, ww = w1 * w1 + w2 * w2;
            const double M = R[R_MPRE] * exp(-ww * R[R_I2T]);
            const double g = M * (pre * (a11 * w1 * w1 + 2.0 * a12 * w1 * w2 + a22 * w2 * w2 +
                                         (q1 * w1 + q2 * w2) * (ww / (2.0 * T) - 2.0)) +
                                  cubic(w1, w2));
            const double pg = (cp[0] + cp[1] * v1 + cp[2] * v2 + cp[3] * (v1 * v1 + v2 * v2)) * M;
            gout[n] = (TS)(g - pg);
        }
    }
}

// Training targets of every cell from the micro solve: (q1, q2, S11, S12, S22, t1, t2) / eps
// with q = (H111 + H122, H112 + H222) / 2, t = (H111 - 3 H122, 3 H112 - H222)
// and S from the g-moments
// gm = eps dv sum (w1^2 - w2^2, 2 w1 w2, |w|^2) G / 2 (entries 4..6).
// With residual = 1 the Navier-Stokes-Fourier values of the cell are
// subtracted; residual = 2 also divides that difference by eps.
// Then the cells with kn <= kn_max that are not next to a non-periodic side are
// appended, in cell order, to (Xo, Yo) from row base (one workgroup; at most
// capacity rows in total); *count receives the new total.
__global__ __launch_bounds__(1024) void k_snapshot2d(const float *__restrict__ feat, const float *__restrict__ kn,
                                                     const uint8_t *__restrict__ edge, const double *__restrict__ H,
                                                     const double *__restrict__ gm, int n, Params P, int residual,
                                                     float kn_max, float *__restrict__ Xo, float *__restrict__ Yo,
                                                     int base, int capacity, int *__restrict__ count)
{
    const double eps = P.eps;
    __shared__ int scan[1024];
    const int per = (n + blockDim.x - 1) / blockDim.x;
    const int c0 = threadIdx.x * per, c1 = min(n, c0 + per);
    int mine = 0;
    for (int c = c0; c < c1; ++c) mine += (!edge[c] && kn[c] <= kn_max);
    scan[threadIdx.x] = mine;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const int v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int pos = base + scan[threadIdx.x] - mine;
    for (int c = c0; c < c1; ++c) {
        if (edge[c] || !(kn[c] <= kn_max)) continue;
        if (pos < capacity) {
            for (int a = 0; a < NF; ++a) Xo[(size_t)pos * NF + a] = feat[(size_t)c * NF + a];
            const double *h = H + 4 * (size_t)c, *m = gm + 7 * (size_t)c;
            double t[NO] = {0.5 * (h[0] + h[2]) / eps, 0.5 * (h[1] + h[3]) / eps, (m[4] + m[6]) / eps, m[5] / eps,
                            (m[6] - m[4]) / eps,          (h[0] - 3.0 * h[2]) / eps, (3.0 * h[1] - h[3]) / eps};
            if (residual) {
                double b[NO];
                nsf_out(feat + (size_t)c * NF, P, b);
                const double f = residual == 2 ? 1.0 / eps : 1.0;
#pragma unroll
                for (int k = 0; k < NO; ++k) t[k] = (t[k] - b[k]) * f;
            }
            float *y = Yo + (size_t)pos * NO;
#pragma unroll
            for (int k = 0; k < NO; ++k) y[k] = (float)t[k];
        }
        ++pos;
    }
    if (threadIdx.x == blockDim.x - 1) *count = min(capacity, base + scan[threadIdx.x]);
}

} // namespace closure

// ------------------------------------------------------------- launchers

namespace closure {

void launch_features2d(const double *Q, const Params &P, float *feat, float *kn, uint8_t *edge, hipStream_t st)
{
    const int n = P.nx * P.ny;
    hipLaunchKernelGGL(k_features2d, dim3((n + 255) / 256), dim3(256), 0, st, Q, P, feat, kn, edge);
}

void launch_cells2d(const double *Q, const Params &P, const MlpDev *w, int residual, float kn_max, uint8_t *cls,
                    float *out, double *H, unsigned long long *nclosure, int *nrebuild, hipStream_t st)
{
    const int n = P.nx * P.ny;
    const dim3 grid((n + 127) / 128), block(256);     // 4 wavefronts x 32 cells
    if (w)
        hipLaunchKernelGGL(k_cells2d<true>, grid, block, 0, st, Q, P, *w, residual, kn_max, cls, out, H, nclosure,
                           nrebuild);
    else
        hipLaunchKernelGGL(k_cells2d<false>, grid, block, 0, st, Q, P, MlpDev{}, 0, kn_max, cls, out, H, nclosure,
                           nrebuild);
}

void launch_mlp_forward(const float *X, int n, const MlpDev &w, float *Y, bool accumulate, float scale,
                        hipStream_t st)
{
    const int ntile = (n + 31) / 32;
    int blocks = (ntile + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, st, X, n, w, Y, accumulate ? 1 : 0, scale);
}

void launch_mlp_grad(const float *X, const float *Y, const int *idx, int first, int count, const MlpDev &w,
                     float *part, float *loss_part, int nwaves, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_grad, dim3(nwaves / 2), dim3(128), 0, st, X, Y, idx, first, count, w, part, loss_part);
}

void launch_mlp_reduce(const float *part, int nparts, const float *loss_part, float *grad, float *loss_acc,
                       int loss_slot, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, nparts, loss_part, grad,
                       loss_acc, loss_slot);
}

void launch_mlp_adam(float *master, float *m1, float *m2, const float *grad, float lr, float b1, float b2, float c1,
                     float c2, float epsa, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, master, m1, m2, grad, lr, b1, b2,
                       c1, c2, epsa);
}

void launch_mlp_pack(const float *master, const MlpDevMut &w, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3((NWP + 255) / 256), dim3(256), 0, st, master, w.W1, w.W2, w.W3, w.Wp, w.b1,
                       w.b2, w.b3);
}

void launch_mlp_norm(const float *X, const float *Y, int n, float *norm, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_norm, dim3(NF + NO), dim3(256), 0, st, X, Y, n, norm);
}

void launch_nsf2d(const float *feat, int n, const Params &P, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_nsf2d, dim3((n + 255) / 256), dim3(256), 0, st, feat, n, P, out);
}

void launch_classify2d(const float *kn, const uint8_t *edge, const float *out, int n, float kn_max, double eps,
                       uint8_t *cls, double *H, unsigned long long *nclosure, int *nrebuild, hipStream_t st)
{
    hipLaunchKernelGGL(k_classify2d, dim3((n + 255) / 256), dim3(256), 0, st, kn, edge, out, n, kn_max, eps, cls, H,
                       nclosure, nrebuild);
}

void launch_rebuild2d(void *G, int g_bytes, const double *rec, const float *out, const uint8_t *cls,
                      const uint8_t *valid, uint8_t *valid_next, int *list, int *nrebuild, const Params &P,
                      hipStream_t st)
{
    const int n = P.nx * P.ny;
    hipLaunchKernelGGL(k_need2d, dim3((n + NEED_BLOCK - 1) / NEED_BLOCK), dim3(NEED_BLOCK), 0, st, cls, valid,
                       valid_next, list, nrebuild, P);
    int blocks = (n + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    if (g_bytes == 8)
        hipLaunchKernelGGL(k_rebuild2d<double>, dim3(blocks), dim3(256), 0, st, (double *)G, rec, out, list, nrebuild,
                           P);
    else
        hipLaunchKernelGGL(k_rebuild2d<float>, dim3(blocks), dim3(256), 0, st, (float *)G, rec, out, list, nrebuild,
                           P);
}

void launch_snapshot2d(const float *feat, const float *kn, const uint8_t *edge, const double *H, const double *gm,
                       int n, const Params &P, int residual, float kn_max, float *Xo, float *Yo, int base,
                       int capacity, int *count, hipStream_t st)
{
    hipLaunchKernelGGL(k_snapshot2d, dim3(1), dim3(1024), 0, st, feat, kn, edge, H, gm, n, P, residual, kn_max,
                       Xo, Yo, base, capacity, count);
}

} // namespace closure
} // namespace mm
