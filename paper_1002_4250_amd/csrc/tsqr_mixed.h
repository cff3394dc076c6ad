// tsqr_mixed.h -- FP64 correction of an FP32 R factor (mixed precision).
//
// Given A (m x n, stored in FP32) and R~, the R factor of A computed by the
// FP32 TSQR path (section 2 of the paper in FP32), one FP64 pass gives R to
// FP64 accuracy when kappa(A) * u32 << 1:
//     Y = A R~^-1   (FP64; kappa(Y) = 1 + O(kappa(A) u32)),
//     G = Y^T Y,    R_c = chol(G) (upper, G = R_c^T R_c),    R = R_c R~.
// This is the second pass of CholeskyQR2 (Fukaya, Nakatsukasa, Yanagisawa and
// Yamamoto, 2014) with the FP32 Householder factorization as the first pass.
// The Cholesky factorization fails (a pivot that is not positive and finite)
// when R~ is too inaccurate; the instance is then flagged, and a batched FP64
// TSQR launch over the FP32 storage, whose workgroups exit at once for
// unflagged instances, refactors it (decided on the device, no host sync).
//
// Two kernels:
//   mixed_gram_kernel   one wavefront per (row block, instance): forward
//                       substitution y = a R~^-1 for one row per lane, then
//                       the rows' contribution to G accumulated in registers,
//                       each lane owning an S x S block of the upper triangle
//                       of G; the block sums go to a workspace slot.
//   mixed_finish_kernel one wavefront per instance: sums the slots in a fixed
//                       order (bit-reproducible), Cholesky with one column per
//                       lane, R = R_c R~, sign-normalized by construction
//                       (both factors have positive diagonals).
#pragma once

#include "tsqr_device.h"
#include "tsqr_internal.h"

namespace tsqr {

namespace dev {

// block index -> (I, J), I <= J, in a 10 x 10 grid
__device__ __forceinline__ void gram_block(int t, int& I, int& J)
{
    I = 0;
    int left = t;
    while (left >= 10 - I) {
        left -= 10 - I;
        ++I;
    }
    J = I + left;
}

// R~ of every instance in FP64, packed by rows ((i, j) at off(i) + j - i, as
// for the leaf triangles), extended by the identity past column n (padding
// columns then solve to 0), followed by the reciprocals of its diagonal.
template <int NC>
__global__ void __launch_bounds__(kWave) mixed_prep_kernel(MixedArgs a)
{
    constexpr int NT = Tri<NC>::kSize;
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    const int n = a.n;
    const float* Rt = a.Rt + (int64_t)b * n * n;
    double* out = a.Rp + (int64_t)b * a.rp_stride;
    for (int idx = lane; idx < NT; idx += kWave) {
        int i = 0;
        while (Tri<NC>::off(i + 1) <= idx) ++i;
        const int j = i + (idx - Tri<NC>::off(i));
        out[idx] = (j < n) ? (double)Rt[i + j * n] : (i == j ? 1.0 : 0.0);
    }
    for (int j = lane; j < NC; j += kWave) out[NT + j] = (j < n) ? 1.0 / (double)Rt[j + j * n] : 1.0;
}

template <int NC>
__global__ void __launch_bounds__(kWave) mixed_gram_kernel(MixedArgs a)
{
    constexpr int S = GramTile<NC>::S;
    constexpr int W = GramTile<NC>::W;
    constexpr int YS = W + 1;                              // LDS row stride of Y
    constexpr int NT = Tri<NC>::kSize;
    __shared__ double Y[kWave * YS];
    const int lane = threadIdx.x;
    const int b = blockIdx.y;
    const int n = a.n;
    // R~ is the same for every lane: read through the scalar unit, so each
    // forward-substitution FMA takes its R~ operand from a scalar register
    const double* __restrict__ Rp = a.Rp + (int64_t)b * a.rp_stride;
    for (int idx = lane; idx < kWave * YS; idx += kWave) Y[idx] = 0.0;
    wave_sync();

    int I = 0, J = 0;
    gram_block(lane < GramTile<NC>::kBlocks ? lane : 0, I, J);
    double acc[S][S];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t < S; ++t) acc[s][t] = 0.0;

    const float* A = a.A + (int64_t)b * a.stride_a;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r1 = (r0 + a.rows_per_block < a.m) ? r0 + a.rows_per_block : a.m;
    // this lane's row of the next 64-row block, loaded one block ahead
    float nxt[NC];
    auto load_rows = [&](int64_t base) {
        const int64_t row = base + lane;
        const bool ok = row < r1;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const bool in = ok && j < n;
            const float v = A[in ? row + (int64_t)j * a.lda : 0];
            nxt[j] = in ? v : 0.0f;
        }
    };
    if (r0 < r1) load_rows(r0);
    for (int64_t base = r0; base < r1; base += kWave) {
        double y[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) y[j] = (double)nxt[j];
        if (base + kWave < r1) load_rows(base + kWave);
        // y := y R~^-1, one row of R~ at a time: after step i, y_i is final
        // and the updates of the step are independent
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double yi = y[i] * Rp[NT + i];
            y[i] = yi;
#pragma unroll
            for (int j = i + 1; j < NC; ++j) y[j] = fmadd(-yi, Rp[Tri<NC>::off(i) + j - i], y[j]);
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) Y[lane * YS + j] = y[j];
        wave_sync();
        if (lane < GramTile<NC>::kBlocks) {
#pragma unroll 8
            for (int r = 0; r < kWave; ++r) {
                double yi[S], yj[S];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    yi[s] = Y[r * YS + I * S + s];
                    yj[s] = Y[r * YS + J * S + s];
                }
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int t = 0; t < S; ++t) acc[s][t] = fmadd(yi[s], yj[t], acc[s][t]);
            }
        }
        wave_sync();
    }
    if (lane < GramTile<NC>::kBlocks) {
        double* out = a.part + ((int64_t)b * a.blocks + blockIdx.x) * (W * W);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int t = 0; t < S; ++t) out[(I * S + s) * W + (J * S + t)] = acc[s][t];
    }
}

template <int NC>
__global__ void __launch_bounds__(kWave) mixed_finish_kernel(MixedArgs a)
{
    constexpr int W = GramTile<NC>::W;
    __shared__ double Rc[NC * NC];       // column-major, ld NC
    __shared__ double Rtl[NC * NC];      // R~ column-major, zero below the diagonal
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    const int n = a.n;
    const float* Rt = a.Rt + (int64_t)b * n * n;
    for (int idx = lane; idx < NC * NC; idx += kWave) {
        const int i = idx % NC, j = idx / NC;
        Rtl[idx] = (i <= j && j < n) ? (double)Rt[i + j * n] : 0.0;
    }
    // column `lane` of G (rows 0..lane), the partial sums added in block order
    double c[NC];
    const double* part = a.part + (int64_t)b * a.blocks * (W * W);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const bool in = i <= lane && lane < n;
        double g = 0.0;
        if (in)
            for (int w = 0; w < a.blocks; ++w) g += part[(int64_t)w * (W * W) + i * W + lane];
        // padding columns: identity, so the factor stays nonsingular
        c[i] = in ? g : ((i == lane && lane >= n) ? 1.0 : 0.0);
    }
    // Cholesky G = Rc^T Rc, column `lane` of Rc in c (rows 0..lane)
    bool good = true;
    static_for<0, NC>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) d = fmadd(bpermute(K << 2, c[i]), c[i], d);
        const double t = c[K] - d;
        const double piv = lane_value(t, K);
        good = good && (piv > 0.0) && (piv < __builtin_inf());
        const double r = __builtin_sqrt(piv);
        c[K] = (lane > K) ? t / r : ((lane == K) ? r : 0.0);
    });
#pragma unroll
    for (int i = 0; i < NC; ++i)
        if (lane < NC) Rc[i + lane * NC] = c[i];
    wave_sync();
    // R = Rc R~, column `lane`: R(i, lane) = sum_{k >= i} Rc(i, k) R~(k, lane)
    double* R = a.R + (int64_t)b * a.ldr * n;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = i; k < NC; ++k) s = fmadd(Rc[i + k * NC], Rtl[k + (lane < NC ? lane : 0) * NC], s);
        if (i < n && lane < n) R[i + (int64_t)lane * a.ldr] = (i <= lane) ? s : 0.0;
    }
    if (lane == 0) {
        a.flags[b] = good ? 0 : 1;
        if (a.flags_out) a.flags_out[b] = good ? 0 : 1;
    }
}

}  // namespace dev
}  // namespace tsqr
