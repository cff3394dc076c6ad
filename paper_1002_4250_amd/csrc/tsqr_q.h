// tsqr_q.h -- the Q factor of TSQR from its stored reflectors.
//
// The leaf+tree kernel in the Q-factor mode keeps every reflector it applies:
// the chunk parts s*x of each leaf's reflectors (V, m x n) with their tau, and
// for every merge of the tree the R2 parts of the operator's reflectors (an
// upper triangle) with their tau (the V and tau outputs of Table 3).  Q is
// then the product of all those reflectors applied to [D; 0], D the signs of
// R's diagonal (R = D R_raw makes Q = Q_raw D), taken in reverse order of
// application:
//   tree pass  (one launch per level, root first): a merge with reflectors
//              H_0..H_{n-1} on the stack [top; bottom] maps the node's n x n
//              block Q_in to H_0 ... H_{n-1} [Q_in; 0]; its top half is the
//              block of the left child, its bottom half that of the right.
//   leaf pass  (one workgroup per leaf, chunks last to first): the chunk's
//              reflectors map the running n x n block T to H_0 ... H_{n-1}
//              [T; 0]; the bottom part is Q's rows of the chunk, the top part
//              the running block for the previous chunk.
// This is the implicit representation of Q that the paper's section 3 notes a
// reduction cannot return, formed explicitly.
#pragma once

#include "tsqr_device.h"
#include "tsqr_internal.h"

namespace tsqr {
namespace dev {

// Level `level` of the tree, root first: workgroup g takes the merge whose
// left operand is leaf g * 2^(level+1).
template <typename T, int NC>
__global__ void __launch_bounds__(kWave) q_tree_kernel(LeafTreeArgs<T> a, int level)
{
    constexpr int NT = Tri<NC>::kSize;
    __shared__ T Vl[NT];
    const int lane = threadIdx.x;
    const int span = 1 << level;
    const int left = blockIdx.x * 2 * span;
    const int right = left + span;
    const int id = left + span - 1;
    for (int i = lane; i < NT; i += kWave) Vl[i] = a.qs.Vn[(int64_t)id * NT + i];
    T* qL = a.qs.qblk + (int64_t)left * NC * NC;
    T* qR = a.qs.qblk + (int64_t)right * NC * NC;
    const T* tau = a.qs.tau_node + (int64_t)id * NC;
    // column `lane` of the stack [top; bottom]: the top block in LDS (one
    // entry per step is touched), the bottom in registers
    __shared__ T Qt[NC * NC + 1];
    for (int i = lane; i < NC * NC; i += kWave) Qt[i] = qL[i];
    T qb[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) qb[i] = T(0);
    wave_sync();
    // reflector J: u = [e_J; v] with v = Vl column J (rows 0..J of the bottom)
    static_for<0, NC>([&](auto jc) {
        constexpr int J = NC - 1 - decltype(jc)::value;
        const int tix = lane < NC ? J + lane * NC : NC * NC;    // lanes past NC: the spare cell
        const T t = tau[J];
        // four partial sums shorten the dependent chain of the dot product
        T wp[4] = {Qt[tix], T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i <= J; ++i) wp[i & 3] = fmadd(Vl[Tri<NC>::off(i) + J - i], qb[i], wp[i & 3]);
        const T w = (wp[0] + wp[1]) + (wp[2] + wp[3]);
        const T tw = t * w;
        Qt[tix] = Qt[tix] - tw;
#pragma unroll
        for (int i = 0; i <= J; ++i) qb[i] = fmadd(-tw, Vl[Tri<NC>::off(i) + J - i], qb[i]);
    });
    wave_sync();
    for (int i = lane; i < NC * NC; i += kWave) qL[i] = Qt[i];
    if (lane < NC) {
#pragma unroll
        for (int i = 0; i < NC; ++i) qR[i + lane * NC] = qb[i];
    }
}

// Q's rows of one leaf: workgroup g takes leaf g.  The chunk rows live in the
// leaf kernel's register layout (lane (q, p): rows p + 16 r of columns 4 s + q);
// the dot products with a reflector go through the same 16 x 17 LDS transpose
// and the coefficients reach the lane rows by DPP row broadcast.
template <typename T, int NC, int RPL>
__global__ void __launch_bounds__(kWave) q_leaf_kernel(LeafTreeArgs<T> a, T* Q, int64_t ldq)
{
    constexpr int CH = 16 * RPL;
    constexpr int NS = Slots<NC>::NS;
    __shared__ T Tq[NC * NC + 1];                // running block, column-major; + a spare cell
    __shared__ T red[kRedElems];
    const int lane = threadIdx.x;
    const int q = lane >> 4, p = lane & 15;
    const int leaf = blockIdx.x;
    const int n = a.n;
    const int64_t r0 = (int64_t)leaf * a.leaf_rows;
    const int64_t r1 = (r0 + a.leaf_rows < a.m) ? r0 + a.leaf_rows : a.m;
    const T* qin = a.qs.qblk + (int64_t)leaf * NC * NC;
    for (int i = lane; i < NC * NC; i += kWave) Tq[i] = qin[i];
    int kcol = 4 * p + q;
    asm volatile("" : "+v"(kcol));
    const bool own = kcol < NC;
    T* rq = red + q * 16 * kRedStride;
    wave_sync();
    if (r1 <= r0) return;
    const int64_t nchunks = (r1 - r0 + CH - 1) / CH;
    for (int64_t t = nchunks - 1; t >= 0; --t) {
        const int64_t cbase = r0 + t * CH;
        const T* tau = a.qs.tau_leaf + (cbase / CH) * NC;
        T c[RPL][NS];
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
            for (int s = 0; s < NS; ++s) c[r][s] = T(0);
        static_for<0, NC>([&](auto jc) {
            constexpr int J = NC - 1 - decltype(jc)::value;
            if (J < n) {
                // V holds every row of the chunk (zero past the end of A)
                const T* vcol = a.qs.V + cbase + p + (int64_t)J * a.qs.ldv;
                T x[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) x[r] = vcol[16 * r];
                const T tj = tau[J];
                static_for<0, NS>([&](auto sc) {
                    constexpr int s = decltype(sc)::value;
                    T acc = x[0] * c[0][s];
#pragma unroll
                    for (int r = 1; r < RPL; ++r) acc = fmadd(x[r], c[r][s], acc);
                    rq[s * kRedStride + p] = acc;
                });
                lds_order();
                T u[16];
                const T* rd = rq + p * kRedStride;
#pragma unroll
                for (int i = 0; i < 16; ++i) u[i] = rd[i];
#pragma unroll
                for (int hh = 8; hh >= 1; hh >>= 1)
#pragma unroll
                    for (int i = 0; i < hh; ++i) u[i] = u[i] + u[i + hh];
                const int tix = own ? J + kcol * NC : NC * NC;
                const T w = Tq[tix] + u[0];
                const T tw = tj * w;
                Tq[tix] = Tq[tix] - tw;
                const T fown = own ? tw : T(0);
                lds_order();
                static_for<0, NS>([&](auto sc) {
                    constexpr int s = decltype(sc)::value;
                    const T f = dpp_mov<0x150 + s>(fown);
#pragma unroll
                    for (int r = 0; r < RPL; ++r) c[r][s] = fmadd(-f, x[r], c[r][s]);
                });
            }
        });
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int64_t row = cbase + p + 16 * r;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int k = 4 * s + q;
                if (row < r1 && k < n) Q[row + (int64_t)k * ldq] = c[r][s];
            }
        }
    }
}

// ---- applying Q^T without forming Q ---------------------------------------------
//
// C = Q^T B (n x k) replays the factorization's reflectors on B in the order
// the factorization applied them to A:
//   leaf pass  (one workgroup per leaf, chunks first to last): the running
//              n x k block T (zero at the start) stacked on the chunk's rows of
//              B is mapped by the chunk's reflectors H_0, ..., H_{n-1} in turn;
//              what is left in the chunk's rows belongs to rows of Q_full^T B
//              past the first n and is dropped.
//   tree pass  (one launch per level, leaves first): a merge maps the stack
//              [T_left; T_right] by its reflectors and keeps the top block.
//   finish     C = D T_root, D the signs the root applied to R.
// k is taken in panels (52 columns in FP64, 64 in FP32); KS column slots
// (4 columns each) are compiled for the panel width and for panels of at most
// 32, 16 and 4 columns.  The per-leaf blocks are kQtCols = 64
// columns wide.

template <typename T, int NC, int RPL, int KS>
__global__ void __launch_bounds__(kWave) qt_leaf_kernel(QtArgs<T> x)
{
    constexpr int CH = 16 * RPL;
    constexpr int KC = 4 * KS;
    __shared__ T Tq[NC * KC + 1];                // running block, column-major ld NC; + a spare cell
    __shared__ T red[kRedElems];
    const LeafTreeArgs<T>& a = x.a;
    const int lane = threadIdx.x;
    const int q = lane >> 4, p = lane & 15;
    const int leaf = blockIdx.x;
    const int n = a.n;
    const int64_t r0 = (int64_t)leaf * a.leaf_rows;
    const int64_t r1 = (r0 + a.leaf_rows < a.m) ? r0 + a.leaf_rows : a.m;
    for (int i = lane; i < NC * KC + 1; i += kWave) Tq[i] = T(0);
    int kcol = 4 * p + q;                        // the column this lane completes
    asm volatile("" : "+v"(kcol));
    const bool own = p < KS;
    T* rq = red + q * 16 * kRedStride;
    wave_sync();
    const int64_t nchunks = r1 > r0 ? (r1 - r0 + CH - 1) / CH : 0;
    for (int64_t t = 0; t < nchunks; ++t) {
        const int64_t cbase = r0 + t * CH;
        const T* tau = a.qs.tau_leaf + (cbase / CH) * NC;
        // the chunk's rows of B in the leaf kernel's register layout
        T c[RPL][KS];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int64_t row = cbase + p + 16 * r;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int col = 4 * s + q;
                c[r][s] = (row < r1 && col < x.k) ? x.B[row + (int64_t)col * x.ldb] : T(0);
            }
        }
        static_for<0, NC>([&](auto jc) {
            constexpr int J = decltype(jc)::value;
            if (J < n) {
                // V holds every row of the chunk (zero past the end of A)
                const T* vcol = a.qs.V + cbase + p + (int64_t)J * a.qs.ldv;
                T xv[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) xv[r] = vcol[16 * r];
                const T tj = tau[J];
                static_for<0, KS>([&](auto sc) {
                    constexpr int s = decltype(sc)::value;
                    T acc = xv[0] * c[0][s];
#pragma unroll
                    for (int r = 1; r < RPL; ++r) acc = fmadd(xv[r], c[r][s], acc);
                    rq[s * kRedStride + p] = acc;
                });
                lds_order();
                T u[16];
                const T* rd = rq + p * kRedStride;
#pragma unroll
                for (int i = 0; i < 16; ++i) u[i] = rd[i];
#pragma unroll
                for (int hh = 8; hh >= 1; hh >>= 1)
#pragma unroll
                    for (int i = 0; i < hh; ++i) u[i] = u[i] + u[i + hh];
                const int tix = own ? J + kcol * NC : NC * KC;
                const T w = Tq[tix] + u[0];
                const T tw = tj * w;
                Tq[tix] = Tq[tix] - tw;
                const T fown = own ? tw : T(0);
                lds_order();
                static_for<0, KS>([&](auto sc) {
                    constexpr int s = decltype(sc)::value;
                    const T f = dpp_mov<0x150 + s>(fown);
#pragma unroll
                    for (int r = 0; r < RPL; ++r) c[r][s] = fmadd(-f, xv[r], c[r][s]);
                });
            }
        });
    }
    wave_sync();
    T* out = x.tq + (int64_t)leaf * NC * kQtCols;
    for (int i = lane; i < NC * KC; i += kWave) out[i] = Tq[i];
}

// Level `level` of the tree, leaves first: workgroup g takes the merge whose
// left operand is leaf g * 2^(level+1); lane j < KC holds column j of the
// bottom block, the top block sits in LDS.
template <typename T, int NC, int KS>
__global__ void __launch_bounds__(kWave) qt_tree_kernel(QtArgs<T> x, int level)
{
    constexpr int NT = Tri<NC>::kSize;
    constexpr int KC = 4 * KS;
    const LeafTreeArgs<T>& a = x.a;
    __shared__ T Vl[NT];
    __shared__ T Tt[NC * KC + 1];
    const int lane = threadIdx.x;
    const int span = 1 << level;
    const int left = blockIdx.x * 2 * span;
    const int right = left + span;
    const int id = left + span - 1;
    for (int i = lane; i < NT; i += kWave) Vl[i] = a.qs.Vn[(int64_t)id * NT + i];
    T* tl = x.tq + (int64_t)left * NC * kQtCols;
    const T* tr = x.tq + (int64_t)right * NC * kQtCols;
    const T* tau = a.qs.tau_node + (int64_t)id * NC;
    for (int i = lane; i < NC * KC; i += kWave) Tt[i] = tl[i];
    T tb[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) tb[i] = lane < KC ? tr[i + lane * NC] : T(0);
    wave_sync();
    // reflector J: u = [e_J; v] with v = Vl column J (rows 0..J of the bottom)
    static_for<0, NC>([&](auto jc) {
        constexpr int J = decltype(jc)::value;
        const int tix = lane < KC ? J + lane * NC : NC * KC;    // lanes past KC: the spare cell
        const T t = tau[J];
        T wp[4] = {Tt[tix], T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i <= J; ++i) wp[i & 3] = fmadd(Vl[Tri<NC>::off(i) + J - i], tb[i], wp[i & 3]);
        const T w = (wp[0] + wp[1]) + (wp[2] + wp[3]);
        const T tw = t * w;
        Tt[tix] = Tt[tix] - tw;
#pragma unroll
        for (int i = 0; i <= J; ++i) tb[i] = fmadd(-tw, Vl[Tri<NC>::off(i) + J - i], tb[i]);
    });
    wave_sync();
    for (int i = lane; i < NC * KC; i += kWave) tl[i] = Tt[i];
}

// C(i, j) = D(i) T_root(i, j) for the k0-th panel of columns, D from the root's
// sign block (the diagonal of the first leaf's Q block).
template <typename T, int NC>
__global__ void __launch_bounds__(kWave) qt_finish_kernel(QtArgs<T> x)
{
    const int n = x.a.n;
    for (int idx = blockIdx.x * kWave + threadIdx.x; idx < n * x.k; idx += gridDim.x * kWave) {
        const int i = idx % n, j = idx / n;
        x.C[i + (int64_t)j * x.ldc] = x.a.qs.qblk[i + i * NC] * x.tq[i + j * NC];
    }
}

}  // namespace dev
}  // namespace tsqr
