// tsqr_mlp.h -- kernels of the learned correction of the sampled
// preconditioner: a GEMM on the BF16 matrix cores with FP32 accumulation, the
// elementwise steps of training a small MLP (bias and ReLU forward and
// backward, bias gradients, the mean-squared-error loss, Adam), and the
// feature, target and correction maps between an R~ and the network.
#pragma once

#include "tsqr_device.h"
#include "tsqr_internal.h"

namespace tsqr {
namespace dev {

// FP32 -> BF16, round to nearest even (a NaN stays a quiet NaN)
__device__ __forceinline__ short bf16_rne(float x)
{
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (short)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// C (M x N, column-major, ldc) = alpha op(A) op(B) + beta C with op(A) M x K
// and op(B) K x N, A and B FP32 in memory (column-major; ta, tb: stored
// transposed), rounded to BF16 as they are loaded and multiplied by the
// 16x16x16 BF16 instruction with FP32 accumulation.  One wavefront per 16 x 16
// tile of C.  The instruction takes A(i, k) from lane l = i + 16 (k / 4),
// element k % 4, B(k, j) from lane j + 16 (k / 4), element k % 4, and returns
// D(i, j) in lane j + 16 (i / 4), element i % 4 (measured on gfx950).  beta = 0
// does not read C.
__global__ void __launch_bounds__(kWave) gemm_bf16_kernel(GemmArgs g)
{
    const int lane = threadIdx.x;
    const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    const int li = lane & 15, lk = 4 * (lane >> 4);
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    const int i = i0 + li, j = j0 + li;
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        bf16x4_t av, bv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + lk + e;
            const bool ina = i < g.M && k < g.K, inb = k < g.K && j < g.N;
            const int64_t ia = g.ta ? k + (int64_t)i * g.lda : i + (int64_t)k * g.lda;
            const int64_t ib = g.tb ? j + (int64_t)k * g.ldb : k + (int64_t)j * g.ldb;
            av[e] = bf16_rne(ina ? g.A[ia] : 0.f);
            bv[e] = bf16_rne(inb ? g.B[ib] : 0.f);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = i0 + lk + r;
        if (row < g.M && j < g.N) {
            float* c = g.C + row + (int64_t)j * g.ldc;
            float v = g.alpha * acc[r];
            if (g.beta != 0.f) v = fmaf(g.beta, *c, v);
            *c = v;
        }
    }
}

// Z(i, j) := act(Z(i, j) + bias(j)) for a rows x cols column-major Z, act the
// identity or ReLU
__global__ void bias_act_kernel(float* Z, int rows, int cols, int64_t ld, const float* bias, int relu)
{
    const int64_t total = (int64_t)rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % rows), j = (int)(t / rows);
        float* z = Z + i + (int64_t)j * ld;
        const float v = *z + bias[j];
        *z = relu ? fmaxf(v, 0.f) : v;
    }
}

// dA(i, j) := dA(i, j) if out(i, j) > 0 else 0 (out: the ReLU's output)
__global__ void relu_grad_kernel(float* dA, const float* out, int rows, int cols, int64_t ld)
{
    const int64_t total = (int64_t)rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % rows), j = (int)(t / rows);
        const int64_t o = i + (int64_t)j * ld;
        if (!(out[o] > 0.f)) dA[o] = 0.f;
    }
}

// s(j) = sum_i Z(i, j), rows added in order (one thread per column)
__global__ void colsum_kernel(const float* Z, int rows, int cols, int64_t ld, float* s)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float acc = 0.f;
    for (int i = 0; i < rows; ++i) acc += Z[i + (int64_t)j * ld];
    s[j] = acc;
}

// D = 2 (Y - T) / (rows cols) and loss = sum (Y - T)^2 / (rows cols), one
// workgroup of 256 threads: thread partial sums in index order, then a fixed
// tree in LDS
__global__ void __launch_bounds__(256) mse_kernel(const float* Y, const float* T, float* D, int rows, int cols,
                                                  int64_t ld, float* loss)
{
    __shared__ float part[256];
    const int64_t total = (int64_t)rows * cols;
    const float scale = 1.f / (float)total;
    float acc = 0.f;
    for (int64_t t = threadIdx.x; t < total; t += 256) {
        const int i = (int)(t % rows), j = (int)(t / rows);
        const int64_t o = i + (int64_t)j * ld;
        const float d = Y[o] - T[o];
        D[o] = 2.f * d * scale;
        acc = fmaf(d, d, acc);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] * scale;
}

// Adam (Kingma and Ba, 2015), step t >= 1: m = b1 m + (1 - b1) g,
// v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        const float gt = g[t];
        const float mt = b1 * m[t] + (1.f - b1) * gt;
        const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
        m[t] = mt;
        v[t] = vt;
        p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    }
}

// The network's input for instance b (R~ FP32, n x n column-major at
// Rt + b n n): X(b, i) = log|R~(i, i)| - mean_k log|R~(k, k)| (i < n) and
// X(b, n - 1 + i) = R~(i - 1, i) / |R~(i - 1, i - 1)| (1 <= i < n); X is
// batch x (2n - 1), column-major with ld = batch.  One thread per instance.
__global__ void surrogate_features_kernel(const float* Rt, int batch, int n, float* X)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const float* R = Rt + (int64_t)b * n * n;
    float mean = 0.f;
    for (int i = 0; i < n; ++i) mean += logf(fabsf(R[i + i * n]));
    mean /= (float)n;
    for (int i = 0; i < n; ++i) X[b + (int64_t)i * batch] = logf(fabsf(R[i + i * n])) - mean;
    for (int i = 1; i < n; ++i)
        X[b + (int64_t)(n - 1 + i) * batch] = R[(i - 1) + i * n] / fabsf(R[(i - 1) + (i - 1) * n]);
}

// Training target for instance b: Y(b, i) = log(|R(i, i)| / |R~(i, i)|) minus
// its mean over i (R the FP64 R of all of A, column-major ld ldr at
// R + b ldr n), batch x n column-major with ld = batch.
__global__ void surrogate_targets_kernel(const double* R, int64_t ldr, const float* Rt, int batch, int n, float* Y)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double* Rb = R + (int64_t)b * ldr * n;
    const float* T = Rt + (int64_t)b * n * n;
    double mean = 0.0;
    for (int i = 0; i < n; ++i) mean += log(fabs(Rb[i + i * ldr]) / fabs((double)T[i + i * n]));
    mean /= (double)n;
    for (int i = 0; i < n; ++i)
        Y[b + (int64_t)i * batch] = (float)(log(fabs(Rb[i + i * ldr]) / fabs((double)T[i + i * n])) - mean);
}

// The largest |log| of a row factor of the correction
constexpr float kMaxLogScale = 1.f;

// The corrected preconditioner: row i of R~ scaled by exp(Y(b, i)), Y clamped
// to [-kMaxLogScale, kMaxLogScale] (a NaN gives the lower bound), so a
// correction can change no row by more than a factor e
__global__ void surrogate_apply_kernel(const float* Rt, const float* Y, int batch, int n, float* Rout)
{
    const int64_t total = (int64_t)batch * n * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t / ((int64_t)n * n));
        const int i = (int)(t % n);
        const float y = fminf(fmaxf(Y[b + (int64_t)i * batch], -kMaxLogScale), kMaxLogScale);
        Rout[t] = Rt[t] * expf(y);
    }
}

}  // namespace dev
}  // namespace tsqr
