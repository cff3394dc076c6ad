// tsqr_inst.hip -- one kernel instantiation of libtsqr.so, selected at compile
// time: -DTSQR_INST_LEAF -DTSQR_INST_TAG=f64|f32 -DTSQR_INST_NC=<n> -DTSQR_INST_RPL=<r>
// for a leaf+tree kernel, -DTSQR_INST_QR with TAG, NC and RPL for the
// Q-factor kernels, -DTSQR_INST_OP with TAG and NC for an operator (and, in
// f64, the mixed-precision) kernels, or -DTSQR_INST_COMMON for the small
// helper kernels.
#include "tsqr_device.h"
#include "tsqr_internal.h"
#include "tsqr_mixed.h"
#include "tsqr_q.h"
#if defined(TSQR_INST_COMMON)
#include "tsqr_mlp.h"  // non-template kernels: defined in this unit only
#endif


namespace tsqr {

#if defined(TSQR_INST_LEAF)
#define TSQR_LEAF_FN(tag, nc, rpl) launch_leaf_tree_##tag##_##nc##_##rpl
#define TSQR_LEAF_FN2(tag, nc, rpl) TSQR_LEAF_FN(tag, nc, rpl)
hipError_t TSQR_LEAF_FN2(TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)(const LeafTreeArgs<TSQR_INST_TAG>& a,
                                                                     hipStream_t s)
{
    // four leaves per workgroup where the leaf count allows: the two lowest
    // tree levels then meet in LDS
    if (a.leaves >= 4 && a.leaves % 4 == 0)
        hipLaunchKernelGGL((dev::tsqr_leaf_tree4_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL>),
                           dim3(a.leaves / 4), dim3(4 * dev::kWave), 0, s, a);
    else
        hipLaunchKernelGGL((dev::tsqr_leaf_tree_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL>), dim3(a.leaves),
                           dim3(dev::kWave), 0, s, a);
    return hipGetLastError();
}
#define TSQR_OCC_FN(tag, nc, rpl) occupancy_leaf_##tag##_##nc##_##rpl
#define TSQR_OCC_FN2(tag, nc, rpl) TSQR_OCC_FN(tag, nc, rpl)
int TSQR_OCC_FN2(TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)()
{
    // every MI355X device runs the same code object: query once per process
    static int cached = -1;
    if (cached < 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, dev::tsqr_leaf_tree_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL>, dev::kWave, 0) !=
            hipSuccess)
            return 0;
        cached = n;
    }
    return cached;
}
#define TSQR_BATCH_FN(tag, nc, rpl) launch_batch_##tag##_##nc##_##rpl
#define TSQR_BATCH_FN2(tag, nc, rpl) TSQR_BATCH_FN(tag, nc, rpl)
hipError_t TSQR_BATCH_FN2(TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)(const BatchArgs<TSQR_INST_TAG>& a, int tiles,
                                                                      hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((dev::tsqr_batch_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL>), dim3(tiles),
                       dim3(dev::kWave), 0, s, a);
    return hipGetLastError();
}
// the FP64 factorization of FP32-stored instances, in the f64 unit at 8 rows per lane
#define TSQR_IS_F64_f64 1
#define TSQR_IS_F64_f32 0
#define TSQR_IS_F64_(tag) TSQR_IS_F64_##tag
#define TSQR_IS_F64(tag) TSQR_IS_F64_(tag)
#if TSQR_IS_F64(TSQR_INST_TAG) && TSQR_INST_RPL == 8
#define TSQR_IN32_FN(nc) launch_batch_f64in32_##nc
#define TSQR_IN32_FN2(nc) TSQR_IN32_FN(nc)
hipError_t TSQR_IN32_FN2(TSQR_INST_NC)(const BatchArgs<double, float>& a, int tiles, hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((dev::tsqr_batch_kernel<double, TSQR_INST_NC, 8, float>), dim3(tiles), dim3(dev::kWave), 0, s,
                       a);
    return hipGetLastError();
}
#endif
#elif defined(TSQR_INST_QR)
#define TSQR_QR_FN(kind, tag, nc, rpl) launch_##kind##_##tag##_##nc##_##rpl
#define TSQR_QR_FN2(kind, tag, nc, rpl) TSQR_QR_FN(kind, tag, nc, rpl)
hipError_t TSQR_QR_FN2(qr_leaf_tree, TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)(
    const LeafTreeArgs<TSQR_INST_TAG>& a, hipStream_t s)
{
    hipLaunchKernelGGL((dev::tsqr_leaf_tree_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL, true>),
                       dim3(a.leaves), dim3(dev::kWave), 0, s, a);
    return hipGetLastError();
}
hipError_t TSQR_QR_FN2(q_tree, TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)(const LeafTreeArgs<TSQR_INST_TAG>& a,
                                                                        int level, int nodes, hipStream_t s)
{
    if (nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL((dev::q_tree_kernel<TSQR_INST_TAG, TSQR_INST_NC>), dim3(nodes), dim3(dev::kWave), 0, s, a,
                       level);
    return hipGetLastError();
}
hipError_t TSQR_QR_FN2(q_leaf, TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)(const LeafTreeArgs<TSQR_INST_TAG>& a,
                                                                        TSQR_INST_TAG* Q, int64_t ldq,
                                                                        hipStream_t s)
{
    hipLaunchKernelGGL((dev::q_leaf_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL>), dim3(a.leaves),
                       dim3(dev::kWave), 0, s, a, Q, ldq);
    return hipGetLastError();
}
// C = Q^T B for one panel of k <= 64 columns: leaf pass, the tree levels
// leaves first, the sign fix
template <int KS>
static hipError_t launch_qt_panel(const QtArgs<TSQR_INST_TAG>& x, int levels, hipStream_t s)
{
    hipLaunchKernelGGL((dev::qt_leaf_kernel<TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL, KS>), dim3(x.a.leaves),
                       dim3(dev::kWave), 0, s, x);
    hipError_t e = hipGetLastError();
    for (int lv = 0; lv < levels && e == hipSuccess; ++lv) {
        const int64_t span = (int64_t)1 << lv;
        const int64_t nodes = x.a.leaves > span ? (x.a.leaves - 1 - span) / (2 * span) + 1 : 0;
        if (nodes <= 0) continue;
        hipLaunchKernelGGL((dev::qt_tree_kernel<TSQR_INST_TAG, TSQR_INST_NC, KS>), dim3((unsigned)nodes),
                           dim3(dev::kWave), 0, s, x, lv);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const int cells = x.a.n * x.k;
    hipLaunchKernelGGL((dev::qt_finish_kernel<TSQR_INST_TAG, TSQR_INST_NC>),
                       dim3((unsigned)((cells + dev::kWave - 1) / dev::kWave)), dim3(dev::kWave), 0, s, x);
    return hipGetLastError();
}
hipError_t TSQR_QR_FN2(qt, TSQR_INST_TAG, TSQR_INST_NC, TSQR_INST_RPL)(const QtArgs<TSQR_INST_TAG>& x, int levels,
                                                                    hipStream_t s)
{
    // panels of 52 columns in FP64 (13 slots of 8 rows stay in registers with
    // the step's working set, no spills), 64 in FP32, so k = n = 50 takes one
    // pass over the reflectors; a narrower panel takes 8, 4 or 1 slots (32, 16
    // or 4 columns): a pass costs a fixed part (reading the reflectors and
    // replaying their chain, about 1.1 ms at 2^22 x 50 in FP64) plus about
    // 0.1 ms per slot
    constexpr int KW = sizeof(TSQR_INST_TAG) == 8 ? 13 : 16;
    if (x.k <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int k0 = 0; k0 < x.k && e == hipSuccess; k0 += 4 * KW) {
        QtArgs<TSQR_INST_TAG> xp = x;
        xp.B = x.B + (int64_t)k0 * x.ldb;
        xp.C = x.C + (int64_t)k0 * x.ldc;
        xp.k = x.k - k0 < 4 * KW ? x.k - k0 : 4 * KW;
        if (xp.k <= 4)
            e = launch_qt_panel<1>(xp, levels, s);
        else if (xp.k <= 16)
            e = launch_qt_panel<4>(xp, levels, s);
        else if (xp.k <= 32)
            e = launch_qt_panel<8>(xp, levels, s);
        else
            e = launch_qt_panel<KW>(xp, levels, s);
    }
    return e;
}
#elif defined(TSQR_INST_OP)
#define TSQR_OP_FN(tag, nc) launch_qr_uppers_##tag##_##nc
#define TSQR_OP_FN2(tag, nc) TSQR_OP_FN(tag, nc)
hipError_t TSQR_OP_FN2(TSQR_INST_TAG, TSQR_INST_NC)(int n, TSQR_INST_TAG* R1, TSQR_INST_TAG* R2,
                                                    TSQR_INST_TAG* tau, hipStream_t s)
{
    hipLaunchKernelGGL((dev::qr_uppers_kernel<TSQR_INST_TAG, TSQR_INST_NC>), dim3(1), dim3(dev::kWave), 0, s, n,
                       R1, R2, tau);
    return hipGetLastError();
}
// the FP64 correction kernels exist once per column count (with the f64 tag)
#define TSQR_MIXED_FN(nc) launch_mixed_##nc
#define TSQR_MIXED_FN2(nc) TSQR_MIXED_FN(nc)
#define TSQR_IS_F64_f64 1
#define TSQR_IS_F64_f32 0
#define TSQR_IS_F64_(tag) TSQR_IS_F64_##tag
#define TSQR_IS_F64(tag) TSQR_IS_F64_(tag)
#if TSQR_IS_F64(TSQR_INST_TAG)
hipError_t TSQR_MIXED_FN2(TSQR_INST_NC)(const MixedArgs& a, int batch, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL((dev::mixed_gram_kernel<TSQR_INST_NC>), dim3(a.blocks, batch),
                       dim3(dev::kGramWaves * dev::kWave), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((dev::mixed_finish_kernel<TSQR_INST_NC>), dim3(batch), dim3(dev::kWave), 0, s, a);
    return hipGetLastError();
}
#endif
#elif defined(TSQR_INST_COMMON)
namespace dev {
__global__ void zero_u32_kernel(unsigned* p, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0u;
}

__global__ void fill_u32_kernel(unsigned* p, int64_t count, unsigned value)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the output function applied to a counter.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Workgroup (k, b) copies block k of instance b's sample: stratum k holds rows
// [k q + min(k, r), ...) of length q + [k < r] (m = nb q + r, nb = s/64), and
// the block of 64 rows starts at a uniform offset in [0, length - 64] drawn
// from splitmix64 of (seed, b, k).  Lane t copies row t of the block, one
// column after another (each wavefront load is 256 contiguous bytes).
__global__ void __launch_bounds__(64) mixed_sample_kernel(SampleArgs a)
{
    const int64_t nb = a.s / kSampleBlock, k = blockIdx.x;
    const int b = blockIdx.y;
    const int64_t q = a.m / nb, r = a.m % nb;
    const int64_t lo = k * q + (k < r ? k : r);
    const int64_t len = q + (k < r ? 1 : 0);
    const uint64_t h = splitmix64(a.seed ^ ((uint64_t)b << 32) ^ (uint64_t)k);
    const int64_t start = lo + (int64_t)(h % (uint64_t)(len - kSampleBlock + 1));
    const int t = threadIdx.x;
    const float* src = a.A + (int64_t)b * a.stride_a + start + t;
    float* dst = a.S + (int64_t)b * a.s * a.n + kSampleBlock * k + t;
    for (int c = 0; c < a.n; ++c) dst[(int64_t)c * a.s] = src[(int64_t)c * a.lda];
}
}  // namespace dev

namespace {
unsigned grid_for(int64_t count, int block)
{
    const int64_t g = (count + block - 1) / block;
    return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}
}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::gemm_bf16_kernel, dim3((unsigned)((g.M + 15) / 16), (unsigned)((g.N + 15) / 16)),
                       dim3(dev::kWave), 0, s, g);
    return hipGetLastError();
}
hipError_t launch_bias_act(float* Z, int rows, int cols, int64_t ld, const float* bias, int relu, hipStream_t s)
{
    hipLaunchKernelGGL(dev::bias_act_kernel, dim3(grid_for((int64_t)rows * cols, 256)), dim3(256), 0, s, Z, rows, cols,
                       ld, bias, relu);
    return hipGetLastError();
}
hipError_t launch_relu_grad(float* dA, const float* out, int rows, int cols, int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(dev::relu_grad_kernel, dim3(grid_for((int64_t)rows * cols, 256)), dim3(256), 0, s, dA, out,
                       rows, cols, ld);
    return hipGetLastError();
}
hipError_t launch_colsum(const float* Z, int rows, int cols, int64_t ld, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(dev::colsum_kernel, dim3(grid_for(cols, 64)), dim3(64), 0, s, Z, rows, cols, ld, out);
    return hipGetLastError();
}
hipError_t launch_mse(const float* Y, const float* T, float* D, int rows, int cols, int64_t ld, float* loss,
                      hipStream_t s)
{
    hipLaunchKernelGGL(dev::mse_kernel, dim3(1), dim3(256), 0, s, Y, T, D, rows, cols, ld, loss);
    return hipGetLastError();
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(dev::adam_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, g, m, v, count, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}
hipError_t launch_surrogate_features(const float* Rt, int batch, int n, float* X, hipStream_t s)
{
    hipLaunchKernelGGL(dev::surrogate_features_kernel, dim3(grid_for(batch, 64)), dim3(64), 0, s, Rt, batch, n, X);
    return hipGetLastError();
}
hipError_t launch_surrogate_targets(const double* R, int64_t ldr, const float* Rt, int batch, int n, float* Y,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(dev::surrogate_targets_kernel, dim3(grid_for(batch, 64)), dim3(64), 0, s, R, ldr, Rt, batch,
                       n, Y);
    return hipGetLastError();
}
hipError_t launch_surrogate_apply(const float* Rt, const float* Y, int batch, int n, float* Rout, hipStream_t s)
{
    hipLaunchKernelGGL(dev::surrogate_apply_kernel, dim3(grid_for((int64_t)batch * n * n, 256)), dim3(256), 0, s, Rt,
                       Y, batch, n, Rout);
    return hipGetLastError();
}

hipError_t launch_mixed_sample(const SampleArgs& a, int batch, hipStream_t s)
{
    if (batch <= 0 || a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::mixed_sample_kernel, dim3((unsigned)(a.s / kSampleBlock), batch), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dev::fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(dev::zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}
#else
#error "select an instantiation with -DTSQR_INST_LEAF, -DTSQR_INST_QR, -DTSQR_INST_OP or -DTSQR_INST_COMMON"
#endif

}  // namespace tsqr
