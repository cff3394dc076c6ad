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
// when R~ is too inaccurate, and R~ is not trusted either when the bound
// ||R_c||_F ||R_c^-1||_F on kappa(A R~^-1) exceeds 1e4; the instance is then
// flagged, and a batched FP64 TSQR launch over the FP32 storage, whose
// workgroups exit at once for unflagged instances, refactors it (decided on
// the device, no host sync).  R~ may also come from the FP32 TSQR of a row
// sample (the sampled plan): the correction is the same.
//
// Two kernels:
//   mixed_gram_kernel   one workgroup of two wavefronts per (row block,
//                       instance), on the FP64 matrix cores: the operand table
//                       of the blocked substitution (below) from R~ into LDS,
//                       then Y = A R~^-1 and the rows' contribution to
//                       G = Y^T Y, 32 rows at a time; the partial G goes to a
//                       workspace slot.
//   mixed_finish_kernel one wavefront per instance: sums the slots in a fixed
//                       order (bit-reproducible), Cholesky with one column per
//                       lane, a bound on kappa(A R~^-1), R = R_c R~,
//                       sign-normalized by construction (both factors have
//                       positive diagonals).
//
// The matrix-core instruction is the 4x4x4 FP64 product with four independent
// blocks, D_b = A_b B_b + C_b (b = 0..3).  Writing lane l as 16 d2 + 4 d1 + d0,
// it takes block d1 of each operand from the lanes with that d1, and
//     A_b(i, k) from lane (d2 = k, d0 = i),  B_b(k, j) from lane (d2 = k, d0 = j),
//     D_b(i, j) to lane (d2 = i, d0 = j)
// (measured on gfx950).  So a result D can be used again as a B operand as it
// stands, and moving it to the contraction position (d2 <-> d0) makes it
// usable as either operand.  The four blocks are four groups of 4 rows of A,
// so one instruction covers 16 rows; every operand below is a 4 x 4 block.
//
// Substitution in transposed form, over the 4-column blocks J of Y = A R~^-1:
//     Z_J^T = A_J^T - sum_{I<J} (R~_IJ)^T Y_I^T,    Y_J^T = (R~_JJ^-1)^T Z_J^T
// (column block J of Y R~ = A, solved with the inverse of the 4 x 4 diagonal
// block: blocked forward substitution, as in a blocked TRSM).  Y_I^T is a D
// result and enters the later updates as their B operand directly; the A
// operands are the constant blocks -(R~_IJ)^T and (R~_JJ^-1)^T.  The updates
// run right-looking (each Y_I^T goes into every later Z_J^T at once), so the
// dependent chain is two instructions per block.  Then every Y_J^T moves its
// rows to the contraction position (a store to LDS at the partner lane's
// index), and
//     G_IJ += (Y_I)^T Y_J      for I <= J,
// one instruction per block pair, accumulated in registers over the row block.
// Each of the two wavefronts substitutes its own 16-row tile and then adds,
// for both tiles, the products of half of the block pairs, so the registers of
// a wavefront hold half of G and two wavefronts fit a SIMD: one's dependent
// substitution chain runs beside the other's independent Gram products.
#pragma once

#include "tsqr_device.h"
#include "tsqr_internal.h"

namespace tsqr {

namespace dev {

// block pairs I <= J in column order
__host__ __device__ constexpr int pair_index(int I, int J) { return J * (J + 1) / 2 + I; }

// block pair p -> (I, J), the inverse of pair_index
__host__ __device__ constexpr int pair_col(int p)
{
    int J = 0;
    while (pair_index(0, J + 1) <= p) ++J;
    return J;
}
__host__ __device__ constexpr int pair_row(int p) { return p - pair_index(0, pair_col(p)); }

// Entry (i, k) of the A operand for block pair p = (I, J), with R~ (FP32,
// column-major, ld n) extended by the identity past column n:
//     I < J:  -R~(4I + k, 4J + i)
//     I = J:  X(k, i),  X = R~_JJ^-1 (4 x 4 upper triangular, by back
//             substitution; a zero pivot gives infinities, and the Cholesky
//             factorization then flags the instance)
__device__ inline double substitution_operand(const float* Rt, int n, int p, int i, int k)
{
    auto rt = [&](int r, int c) -> double {
        if (r > c) return 0.0;
        return (c < n) ? (double)Rt[r + (int64_t)c * n] : (r == c ? 1.0 : 0.0);
    };
    const int J = pair_col(p), I = p - pair_index(0, J);
    if (I < J) return -rt(4 * I + k, 4 * J + i);
    // column i of X = U^-1, U = R~_JJ: X(i, i) = 1/U(i, i) and, upward,
    // X(r, i) = -(sum_{q=r+1..i} U(r, q) X(q, i)) / U(r, r)
    const int c0 = 4 * J;
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    x[i] = 1.0 / rt(c0 + i, c0 + i);
    for (int r = i - 1; r >= 0; --r) {
        double t = 0.0;
        for (int q = r + 1; q <= i; ++q) t += rt(c0 + r, c0 + q) * x[q];
        x[r] = -t / rt(c0 + r, c0 + r);
    }
    return x[k];
}

__device__ __forceinline__ double mfma4(double a, double b, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramWaves = 2;

// The work of one wavefront of the Gram kernel: the substitution of its own
// tile in every iteration and, for both tiles of the iteration, the products
// of block pairs [P0, P1).
template <int NC, int P0, int P1>
__device__ __forceinline__ void gram_wave(const MixedArgs& a, const double* opl,
                                          double (&ys)[2][kGramWaves][MfmaGram<NC>::NB][kWave], int wave)
{
    constexpr int NB = MfmaGram<NC>::NB;
    constexpr int W = MfmaGram<NC>::W;
    constexpr int NQ = P1 - P0;
    const int lane = threadIdx.x & (kWave - 1);
    const int d0 = lane & 3, d1 = (lane >> 2) & 3, d2 = lane >> 4;
    const int b = blockIdx.y;
    const int n = a.n;
    // (the LDS offset passes through an opaque copy every iteration, so the
    // compiler reads each operand where it is used instead of hoisting all of
    // them into registers)
    int lofs = 4 * d0 + d2;
    auto opnd = [&](int p) -> double { return opl[p * 16 + lofs]; };
    double g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = 0.0;

    const float* A = a.A + (int64_t)b * a.stride_a;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r1 = (r0 + a.rows_per_block < a.m) ? r0 + a.rows_per_block : a.m;
    // Lane (d2, d1, d0) holds row 4 d1 + d0 of a 16-row tile in column 4J + d2
    // of block J: the D layout of Z_J^T.  Columns past n read column n - 1
    // instead (no select in the loop): they only reach padding columns of Y
    // and padding entries of G, since R~ is the identity there and its
    // off-diagonal blocks are zero in padding rows, and the finish kernel never
    // reads those entries.  Block J is read from the uniform column 4 jc(J),
    // jc(J) = min(J, jl) with jl = (n - 1)/4, at the per-lane offset of
    // (column - 4 jc(J)) in [0, 3]: d2 for J < jl, eb from jl on.  Rows past
    // the row block read as zero.
    const int trow = 4 * d1 + d0;
    const int tdst = 16 * d0 + 4 * d1 + d2;     // the d2 <-> d0 partner
    const int jl = (n - 1) >> 2;
    const int eb = ((4 * jl + d2 < n) ? 4 * jl + d2 : n - 1) - 4 * jl;
    const int64_t offa = trow + (int64_t)d2 * a.lda;
    const int64_t offb = trow + (int64_t)eb * a.lda;
    auto load_tile = [&](float (&dst)[NB], int64_t base) {
        const bool ok = base + trow < r1;
#pragma unroll
        for (int J = 0; J < NB; ++J) {
            const int jc = J < jl ? J : jl;
            const float* __restrict__ colp = A + base + (int64_t)(4 * jc) * a.lda;
            const float v = colp[J < jl ? offa : offb];
            dst[J] = ok ? v : 0.0f;
        }
    };
    // An iteration takes kGramWaves * 16 rows: wave w substitutes the tile at
    // base + 16 w (rows past r1 are zero and add nothing), every tile's Y^T goes
    // to LDS, and each wave adds every tile's products for its block pairs.
    // Tiles are loaded two iterations ahead (two register buffers, the loop
    // unrolled by two), which keeps enough loads in flight to cover the memory
    // latency.
    constexpr int64_t STEP = kGramWaves * 16;
    int buf = 0;
    auto iteration = [&](float (&cur)[NB], int64_t base) {
        asm volatile("" : "+v"(lofs));
        double z[NB];
#pragma unroll
        for (int J = 0; J < NB; ++J) z[J] = (double)cur[J];
        if (base + 2 * STEP < r1) load_tile(cur, base + 2 * STEP + 16 * wave);
        static_for<0, NB>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            z[I] = mfma4(opnd(pair_index(I, I)), z[I], 0.0);          // Y_I^T
            static_for<I + 1, NB>([&](auto jc) {
                constexpr int J = decltype(jc)::value;
                z[J] = mfma4(opnd(pair_index(I, J)), z[I], z[J]);     // Z_J^T -= (R~_IJ)^T Y_I^T
            });
        });
#pragma unroll
        for (int I = 0; I < NB; ++I) ys[buf][wave][I][tdst] = z[I];
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kGramWaves; ++w) {
            double t[NB];
#pragma unroll
            for (int I = 0; I < NB; ++I) t[I] = ys[buf][w][I][lane];
            static_for<0, NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                g[q] = mfma4(t[pair_row(P0 + q)], t[pair_col(P0 + q)], g[q]);
            });
        }
        buf ^= 1;
    };
    float nx0[NB], nx1[NB];
    if (r0 < r1) load_tile(nx0, r0 + 16 * wave);
    if (r0 + STEP < r1) load_tile(nx1, r0 + STEP + 16 * wave);
    for (int64_t base = r0; base < r1; base += 2 * STEP) {
        iteration(nx0, base);
        if (base + STEP < r1) iteration(nx1, base + STEP);
    }
    // the four row groups (instruction blocks, d1) hold partial sums of every
    // block of G: add them within each 16-lane row, then the lanes with d1 = 0
    // write block (I, J) of the upper block triangle, entry (d2, d0)
    double* out = a.part + ((int64_t)b * a.blocks + blockIdx.x) * (W * W);
    static_for<0, NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        double v = g[q];
        v = v + dpp_mov<0x124>(v);    // row_ror:4
        v = v + dpp_mov<0x128>(v);    // row_ror:8
        if (d1 == 0) out[(4 * pair_row(P0 + q) + d2) * W + 4 * pair_col(P0 + q) + d0] = v;
    });
}

template <int NC>
__global__ void __launch_bounds__(kGramWaves * kWave) mixed_gram_kernel(MixedArgs a)
{
    constexpr int NB = MfmaGram<NC>::NB;
    constexpr int NP = MfmaGram<NC>::NP;
    constexpr int Q = (NP + kGramWaves - 1) / kGramWaves;
    // the operand table, entry (i, k) of pair p at 16 p + 4 i + k
    __shared__ double opl[NP * 16];
    // Y^T blocks of the two tiles of an iteration (one per wave), stored at the
    // contraction position (lane (d2, d1, d0) writes where lane (d0, d1, d2)
    // reads), double-buffered across iterations
    __shared__ double ys[2][kGramWaves][NB][kWave];
    const int b = blockIdx.y;
    const float* Rt = a.Rt + (int64_t)b * a.n * a.n;
    for (int idx = threadIdx.x; idx < NP * 16; idx += kGramWaves * kWave)
        opl[idx] = substitution_operand(Rt, a.n, idx >> 4, (idx >> 2) & 3, idx & 3);
    __syncthreads();
    // wave w owns block pairs [w Q, (w + 1) Q)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    static_for<0, kGramWaves>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        constexpr int P0 = w * Q < NP ? w * Q : NP;
        constexpr int P1 = (w + 1) * Q < NP ? (w + 1) * Q : NP;
        if (wave == w) gram_wave<NC, P0, P1>(a, opl, ys, w);
    });
}

// bound on ||Rc||_F ||Rc^-1||_F (>= kappa_2(A R~^-1)) for a trusted correction;
// an FP32 R~ of a matrix with kappa(A) <= 1e8 gives about n (1 + kappa(A) 2^-24)
constexpr double kMaxKappaY = 1e4;

template <int NC>
__global__ void __launch_bounds__(kWave) mixed_finish_kernel(MixedArgs a)
{
    constexpr int W = MfmaGram<NC>::W;
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
    // column `lane` of G (rows 0..lane), the partial sums added in block order;
    // a slot's NC loads are issued together (entries below the diagonal
    // block triangle are never written and are discarded below)
    double c[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) c[i] = 0.0;
    const double* part = a.part + (int64_t)b * a.blocks * (W * W) + (lane < n ? lane : 0);
    for (int w = 0; w < a.blocks; ++w) {
#pragma unroll
        for (int i = 0; i < NC; ++i) c[i] += part[(int64_t)w * (W * W) + i * W];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        // padding columns: identity, so the factor stays nonsingular
        const bool in = i <= lane && lane < n;
        c[i] = in ? c[i] : ((i == lane && lane >= n) ? 1.0 : 0.0);
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
    // Y = A R~^-1 = Q Rc, so kappa_2(Y) = kappa_2(Rc) <= ||Rc||_F ||Rc^-1||_F.
    // Past kMaxKappaY the correction is not trusted (its Gram matrix carries
    // a relative error of order kappa(Y)^2 u in its smallest directions) and
    // the instance takes the FP64 path as well.  Column `lane` of X = Rc^-1 by
    // back substitution against the rows of Rc in LDS; padding columns are
    // left out of both norms.
    {
        double sr = 0.0, sx = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) sr = fmadd(c[i], c[i], sr);
        double x[NC];
#pragma unroll
        for (int i = NC - 1; i >= 0; --i) {
            double t = (i == lane) ? 1.0 : 0.0;
#pragma unroll
            for (int k = i + 1; k < NC; ++k) t = fmadd(-Rc[i + k * NC], x[k], t);
            x[i] = (i <= lane) ? t / Rc[i + i * NC] : 0.0;
            sx = fmadd(x[i], x[i], sx);
        }
        if (lane >= n) sx = sr = 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            sx += __shfl_xor(sx, off);
            sr += __shfl_xor(sr, off);
        }
        good = good && (sr * sx <= kMaxKappaY * kMaxKappaY);
    }
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
