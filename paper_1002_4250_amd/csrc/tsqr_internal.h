// tsqr_internal.h -- declarations shared by the C-ABI layer and the kernel
// instantiation units of libtsqr.so (the public interface is include/tsqr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsqr_instances.h"

namespace tsqr {

// Reflector storage of the Q-factor mode (unused by the R-only kernels).
template <typename T>
struct QStore {
    T* V;                 // (chunks x chunk rows) x n, leading dimension ldv: the chunk part s*x of
                          // every leaf reflector, zero in the rows of a last chunk past the end of A
    int64_t ldv;
    T* tau_leaf;          // (global chunk index) x NC
    T* Vn;                // per tree node (counter id): packed NC x NC triangle, the R2 part of its reflectors
    T* tau_node;          // per tree node: NC
    T* qblk;              // per leaf: NC x NC column-major block of Q (output of the tree pass)
};

// T is the arithmetic type; TIn the storage type of A (FP32 storage factored
// in FP64 for the mixed-precision fallback; T otherwise).
template <typename T, typename TIn = T>
struct LeafTreeArgs {
    const TIn* A;         // m-by-n, column-major
    int64_t m;
    int64_t lda;
    int n;
    int64_t leaf_rows;    // rows per leaf (multiple of the chunk)
    int leaves;           // P = ceil(m / leaf_rows), at least 1
    T* tri;               // workspace: P packed triangles
    unsigned* tickets;    // workspace: P tree counters, zero on entry and on exit
    T* R;                 // n-by-n output
    int64_t ldr;
    QStore<T> qs;         // Q-factor mode only
    uint64_t* stamps = nullptr;  // null, or per leaf: start, leaf phase done, exit, level stopped at (+100: root)
};

// Batched execution: per-instance description and the (instance, leaf) tiles.
struct BatchInstance {
    int64_t a_off;        // element offset of the instance's matrix in A
    int64_t m;
    int64_t lda;
    int64_t leaf_rows;
    int64_t tri_off;      // element offset of its first triangle slot in tri
    int64_t ticket_off;   // index of its first tree counter
    int32_t leaves;
    int32_t pad;
};

struct BatchTile {
    int32_t inst;
    int32_t leaf;
};

template <typename T, typename TIn = T>
struct BatchArgs {
    const TIn* A;
    const int* run_if;           // null, or per instance: factor it only where run_if[b] != 0
    int n;
    const BatchInstance* inst;   // device table
    const BatchTile* tiles;      // device table, one per workgroup
    T* tri;
    unsigned* tickets;
    T* R;                        // instance b's R at R + b * ldr * n
    int64_t ldr;
    uint64_t* stamps = nullptr;  // null, or per workgroup: (start, end) on the device's constant-rate clock
};

using f64 = double;
using f32 = float;

#define TSQR_DECLARE_LEAF(tag, NC, RPL) \
    hipError_t launch_leaf_tree_##tag##_##NC##_##RPL(const LeafTreeArgs<tag>& a, hipStream_t s);
#define TSQR_DECLARE_OCC(tag, NC, RPL) int occupancy_leaf_##tag##_##NC##_##RPL();
#define TSQR_DECLARE_BATCH(tag, NC, RPL) \
    hipError_t launch_batch_##tag##_##NC##_##RPL(const BatchArgs<tag>& a, int tiles, hipStream_t s);
#define TSQR_DECLARE_OP(tag, NC) \
    hipError_t launch_qr_uppers_##tag##_##NC(int n, tag* R1, tag* R2, tag* tau, hipStream_t s);
TSQR_LEAF_INSTANCES(TSQR_DECLARE_LEAF)
TSQR_LEAF_INSTANCES(TSQR_DECLARE_BATCH)
TSQR_LEAF_INSTANCES(TSQR_DECLARE_OCC)
TSQR_OP_INSTANCES(TSQR_DECLARE_OP)
// the FP64 factorization of FP32-stored instances (mixed-precision fallback),
// one per column count at 8 rows per lane
#define TSQR_DECLARE_BATCH_IN32(NC) \
    hipError_t launch_batch_f64in32_##NC(const BatchArgs<double, float>& a, int tiles, hipStream_t s);
TSQR_DECLARE_BATCH_IN32(16)
TSQR_DECLARE_BATCH_IN32(32)
TSQR_DECLARE_BATCH_IN32(50)
TSQR_DECLARE_BATCH_IN32(64)
#undef TSQR_DECLARE_BATCH_IN32
#undef TSQR_DECLARE_LEAF
#undef TSQR_DECLARE_BATCH
#undef TSQR_DECLARE_OCC
#undef TSQR_DECLARE_OP

hipError_t launch_zero_u32(unsigned* p, int64_t count, hipStream_t s);

// Row sample of every instance for the sampled preconditioner: blocks of
// kSampleBlock contiguous rows, one block drawn uniformly inside each of
// s/kSampleBlock equal strata of the m rows, copied to S (instance b's s x n
// sample at S + b*s*n, column-major, ld s).  s is a multiple of kSampleBlock
// with kSampleBlock <= s < m.
constexpr int kSampleBlock = 64;
struct SampleArgs {
    const float* A;
    int64_t m, lda, stride_a;
    int n;
    float* S;
    int64_t s;
    uint64_t seed;
};
hipError_t launch_mixed_sample(const SampleArgs& a, int batch, hipStream_t s);

// The learned correction of the sampled preconditioner (tsqr_mlp.h).
struct GemmArgs {
    int ta, tb;
    int M, N, K;
    float alpha, beta;
    const float* A;
    int64_t lda;
    const float* B;
    int64_t ldb;
    float* C;
    int64_t ldc;
};
hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s);
hipError_t launch_bias_act(float* Z, int rows, int cols, int64_t ld, const float* bias, int relu, hipStream_t s);
hipError_t launch_relu_grad(float* dA, const float* out, int rows, int cols, int64_t ld, hipStream_t s);
hipError_t launch_colsum(const float* Z, int rows, int cols, int64_t ld, float* out, hipStream_t s);
hipError_t launch_mse(const float* Y, const float* T, float* D, int rows, int cols, int64_t ld, float* loss,
                      hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_surrogate_features(const float* Rt, int batch, int n, float* X, hipStream_t s);
hipError_t launch_surrogate_targets(const double* R, int64_t ldr, const float* Rt, int batch, int n, float* Y,
                                    hipStream_t s);
hipError_t launch_surrogate_apply(const float* Rt, const float* Y, int batch, int n, float* Rout, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned value, hipStream_t s);

// Applying Q^T from the stored reflectors: B (m x k, column-major, ldb), the
// per-leaf NC x kQtCols blocks tq (column-major, ld NC), the output C (n x k,
// ldc).
constexpr int kQtCols = 64;
template <typename T>
struct QtArgs {
    LeafTreeArgs<T> a;
    const T* B;
    int64_t ldb;
    int k;
    T* tq;
    T* C;
    int64_t ldc;
};

// Q-factor mode (FP64): the leaf+tree kernel storing its reflectors, one
// launch per tree level top-down, then one pass over the leaves.
#define TSQR_QR_INSTANCES_DECL(tag, NC, RPL)                                                          \
    hipError_t launch_qr_leaf_tree_##tag##_##NC##_##RPL(const LeafTreeArgs<tag>& a, hipStream_t s);  \
    hipError_t launch_q_tree_##tag##_##NC##_##RPL(const LeafTreeArgs<tag>& a, int level, int nodes,   \
                                                   hipStream_t s);                                    \
    hipError_t launch_q_leaf_##tag##_##NC##_##RPL(const LeafTreeArgs<tag>& a, tag* Q, int64_t ldq,    \
                                                   hipStream_t s);                                    \
    hipError_t launch_qt_##tag##_##NC##_##RPL(const QtArgs<tag>& x, int levels, hipStream_t s);
TSQR_QR_INSTANCES(TSQR_QR_INSTANCES_DECL)
#undef TSQR_QR_INSTANCES_DECL

// The FP64 correction on the matrix cores works on 4-column blocks (the
// 4x4x4 FP64 instruction with four independent blocks): NB blocks cover the
// padded width W = 4 NB >= NC, and NP block pairs I <= J make up the block
// upper triangle of R~ and of G.
template <int NC>
struct MfmaGram {
    static constexpr int NB = (NC + 3) / 4;
    static constexpr int W = 4 * NB;
    static constexpr int NP = NB * (NB + 1) / 2;
};

struct MixedArgs {
    const float* A;        // instance b at A + b * stride_a, column-major, lda
    int64_t m;
    int64_t lda;
    int64_t stride_a;
    int n;
    const float* Rt;       // R~ of instance b at Rt + b * n * n, column-major, ld n
    double* part;          // per (instance, row block): W x W partial Gram sums
    int64_t rows_per_block;  // a multiple of 16
    int blocks;            // row blocks per instance
    double* R;             // instance b's R at R + b * ldr * n
    int64_t ldr;
    int* flags;            // per instance: 0 corrected, 1 Cholesky failed
    int* flags_out;        // null, or the caller's copy of flags
};

#define TSQR_DECLARE_MIXED(NC) hipError_t launch_mixed_##NC(const MixedArgs& a, int batch, hipStream_t s);
TSQR_DECLARE_MIXED(16)
TSQR_DECLARE_MIXED(32)
TSQR_DECLARE_MIXED(50)
TSQR_DECLARE_MIXED(64)
#undef TSQR_DECLARE_MIXED

}  // namespace tsqr
