// tsqr_device.h -- gfx950 device code for the R factor of a tall-skinny matrix
// by Householder TSQR (Langou, arXiv:1002.4250, sections 2-3).
//
// Execution model (one wavefront of 64 lanes per workgroup):
//   * A leaf is a contiguous block of rows of A.  Its wavefront keeps the n-by-n
//     triangle R in LDS (packed by rows) and streams the block through
//     registers in chunks of 16*RPL rows.  Each chunk C is merged into R by
//     R := R-factor of [R; C]: for every column j one Householder reflector
//     built from R(j,j) and C(:,j) is applied to the trailing columns (the
//     structured update of Table 3 with R2 replaced by a dense chunk: a flat
//     tree inside the leaf; section 2 allows any tree).
//   * Leaves then combine with the paper's operator qr(R1, R2) over a binary
//     tree pairing leaf i with i + 2^level (lower index on top), the merge done
//     by whichever wavefront of the pair arrives last (atomic ticket), so no
//     wavefront ever waits on another.  A merge has only NC rows, so it uses a
//     second layout: one column of R2 per lane (merge_columns).  Workgroups
//     are numbered onto leaves so that tree siblings share an XCD and its L2
//     (xcd_local_leaf).
//   * The root flips rows with a negative diagonal (section 2's positive
//     diagonal convention) and writes R.
//
// Register layout of a chunk: the wavefront is four 16-lane rows q = 0..3.
// Lane (q, p) = lane 16q + p holds chunk rows p + 16r (r < RPL) of the
// columns k = 4s + q (slot s < NS = ceil(NC/4)): the columns are dealt
// cyclically to the four lane rows, the matrix rows to the 16 lanes of a lane
// row.  A dot product over the chunk's rows is then a sum over RPL registers
// and over only 16 lanes, which goes through LDS in one transpose (each lane
// adds 16 values); the pivot column reaches all lane rows by one ds_bpermute
// per register, and each column's update coefficient reaches its lane row by
// a DPP row broadcast.
//
// Per Householder step j (x = C(:,j), k > j the trailing columns):
//     sigma^2 = x.x,  d_k = x.C(:,k)
//     beta = -sign(alpha) sqrt(alpha^2 + sigma^2), alpha = R(j,j)
//     tau = (beta - alpha)/beta, s = 1/(alpha - beta)        (v = s x)
//     w_k = R(j,k) + s d_k,  R(j,k) -= tau w_k,  C(:,k) -= (tau s w_k) x
// which is the reflector generation and rank-1 update of Table 3 with the
// Householder vector kept unscaled (v = s x) so that no lane has to rescale
// its rows before the dot products.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>
#include <utility>

#include "tsqr_internal.h"

namespace tsqr {
namespace dev {

constexpr int kWave = 64;
constexpr int kRedStride = 17;                  // odd stride: conflict-free LDS transpose
constexpr int kRedElems = 4 * 16 * kRedStride;  // one 16 x 17 tile per lane row

template <int NC>
struct Tri {
    static constexpr int kSize = NC * (NC + 1) / 2;
    // LDS copies get one wavefront of padding: a spare cell for branch-free
    // writes and room for column reads of lanes past the triangle
    static constexpr int kPadded = kSize + 64;
    // packed row-major upper triangle: row j starts at off(j), entry (j,k) at off(j)+k-j
    static constexpr __host__ __device__ int off(int j) { return j * NC - (j * (j - 1)) / 2; }
};

// The leaf's reduction tiles and, in the tree, the partner's triangle share
// one LDS buffer: they are never live at the same time.
template <int NC>
struct LdsScratch {
    static constexpr int kElems = kRedElems > Tri<NC>::kPadded ? kRedElems : Tri<NC>::kPadded;
};

template <int NC>
struct Slots {
    static constexpr int NS = (NC + 3) / 4;     // column slots per lane
};

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(static_cast<F&&>(f));
    }
}

template <typename T> struct Limits;
template <> struct Limits<double> { static constexpr double tiny = 2.2250738585072014e-308; };
template <> struct Limits<float> { static constexpr float tiny = 1.17549435e-38f; };

// ---- cross-lane primitives -------------------------------------------------

// Row rotations read a valid lane in every row, so no "old" value is needed.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x)
{
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Sum over the 16 lanes of each lane row, returned in all 16 (bit-identical).
template <typename T>
__device__ __forceinline__ T row_allreduce16(T x)
{
    x = x + dpp_mov<0x128>(x);   // row_ror:8
    x = x + dpp_mov<0x124>(x);   // row_ror:4
    x = x + dpp_mov<0x122>(x);   // row_ror:2
    x = x + dpp_mov<0x121>(x);   // row_ror:1
    return x;
}

// Fused multiply-add and absolute value in the element type (the generic
// builtins would take float operands through double).
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }

// Value of x held by the lane whose byte address (4 * lane) is src.
__device__ __forceinline__ double bpermute(int src, double x)
{
    int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(x));
    int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bpermute(int src, float x)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(x)));
}

// Value of x in lane `l` (l uniform), for every lane.
__device__ __forceinline__ double lane_value(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// Orders this wavefront's LDS accesses around a point without constraining
// arithmetic: LDS operations of one wavefront execute in order, so only the
// compiler has to be kept from moving them across.
// This thread's lane in its wavefront (workgroups may hold several)
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ void lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- reflector scalars ---------------------------------------------------------

// With S = alpha^2 + sigma^2, nrm = sqrt(S) and sgn = sign(alpha) read from its
// sign bit:
//     beta = -sgn nrm,  tau = (beta - alpha)/beta = (|alpha| + nrm)/nrm,
//     s = 1/(alpha - beta) = sgn/(|alpha| + nrm),  tau*s = sgn/nrm.
// 1/nrm comes from the hardware reciprocal square root refined by two Newton
// steps, nrm = S/sqrt(S) with one Newton correction, 1/(|alpha| + nrm) from the
// hardware reciprocal with two Newton steps: a short dependent chain instead
// of two IEEE divisions and a square root.  (The FP64 hardware estimates are
// good to about 2^-24 on gfx950; one quadratic step leaves errors of tens of
// ulps, two reach the rounding level.)  A column whose sigma^2 is below
// the smallest normal number gives the identity reflector.
template <typename T>
struct Reflector {
    T beta, tau, s, ts;
};

__device__ __forceinline__ double hw_rsq(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double hw_rcp(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ Reflector<T> make_reflector(T alpha, T sigma2)
{
    const T S = fmadd(alpha, alpha, sigma2);
    T y = hw_rsq(S);
    const T hS = T(0.5) * S;
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fmadd(y, fmadd(-hS * y, y, T(0.5)), y);
    T nrm = S * y;
    nrm = fmadd(T(0.5) * y, fmadd(-nrm, nrm, S), nrm);
    const T d = absv(alpha) + nrm;
    T q = hw_rcp(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) q = fmadd(q, fmadd(-d, q, T(1)), q);
    const bool neg = __builtin_signbit(alpha);
    const bool ok = sigma2 >= Limits<T>::tiny;
    Reflector<T> r;
    r.beta = ok ? (neg ? nrm : -nrm) : alpha;
    r.tau = ok ? d * y : T(0);
    r.s = ok ? (neg ? -q : q) : T(0);
    r.ts = ok ? (neg ? -y : y) : T(0);
    return r;
}

// ---- one Householder step of a leaf -------------------------------------------

// Where a leaf prefetches its next chunk from.  A register slot holds four
// columns (one per lane row); once its four columns are finished (after step
// 4s+3) the whole slot is refilled with the next chunk's columns 4s..4s+3 by
// one wavefront-wide load per register, into registers no later step of the
// current chunk reads, so no step waits for the loads.  `col` is a per-lane
// running pointer to (row base + p, column 4s + q) of the next slot; lda and n
// pass through an opaque register copy so the compiler keeps that one pointer
// instead of precomputing one address per slot.
//
// The loads are branch-free: a lane whose column lies past n reads from a
// block of zeros instead, so in a chunk whose rows all lie inside the leaf
// (every chunk but a ragged last one) each register is one load at a constant
// offset.  Only a ragged chunk selects per row.  `state` is uniform: 0 no next
// chunk, 1 full chunk, 2 ragged chunk.
static __device__ double kZerosF64[256];
static __device__ float kZerosF32[256];
__device__ __forceinline__ const double* zeros_for(const double*) { return kZerosF64; }
__device__ __forceinline__ const float* zeros_for(const float*) { return kZerosF32; }

template <typename T, int RPL, typename TIn = T>
struct Prefetch {
    const TIn* col;      // per lane: &A(base + p, 4s + q) for the next slot s to fill
    const TIn* zero;     // per lane: zero block + p
    int64_t lda4;        // uniform: 4 * lda
    int cols_left;       // per lane: n - (4s + q)
    int state;           // uniform: 0 none, 1 full chunk, 2 ragged chunk
    int rows;            // uniform: rows of the next chunk inside the leaf
};

template <typename T, int RPL, typename TIn = T>
__device__ __forceinline__ Prefetch<T, RPL, TIn> make_prefetch(const TIn* A, int64_t lda, int n, int64_t base,
                                                               int64_t r1, int q, int p)
{
    static_assert(16 * RPL <= 256, "zero block too small");
    Prefetch<T, RPL, TIn> pf;
    int64_t ld = lda;
    int nn = n;
    asm volatile("" : "+s"(ld), "+s"(nn));
    pf.col = A + (base < r1 ? base : 0) + p + (int64_t)q * ld;
    pf.zero = zeros_for(A) + p;
    pf.lda4 = 4 * ld;
    pf.cols_left = nn - q;
    const int64_t left = r1 - base;
    pf.state = left <= 0 ? 0 : (left >= 16 * RPL ? 1 : 2);
    pf.rows = left <= 0 ? 0 : (left >= 16 * RPL ? 16 * RPL : (int)left);
    return pf;
}

// Fill register slot `slot` with the next chunk's columns and advance.
template <typename T, int RPL, int NS, typename TIn>
__device__ __forceinline__ void prefetch_slot(T (&c)[RPL][NS], int slot, Prefetch<T, RPL, TIn>& pf, int p)
{
    if (pf.state != 0) {
        const TIn* ptr = pf.cols_left > 0 ? pf.col : pf.zero;
        if (pf.state == 1) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) c[r][slot] = (T)ptr[16 * r];
        } else {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const bool ok = p + 16 * r < pf.rows;
                c[r][slot] = (T)*(ok ? ptr + 16 * r : pf.zero + 16 * r);
            }
        }
    }
    pf.col += pf.lda4;
    pf.cols_left -= 4;
}

// Where a leaf in the Q-factor mode writes the reflectors of its current
// chunk: column J of V gets the chunk part s*x of reflector J, tau[J] its tau.
// V has a row for every row of every chunk, so the rows of a partial last
// chunk past the end of A (whose entries are zero) are stored like the others.
template <typename T>
struct VSink {
    T* V;
    int64_t ldv;
    T* tau;
    int64_t cbase;    // first row of the chunk
    int n;
};

// Step J of R := qr([R; C]) with R packed in LDS (Rs) and C in registers.  The
// NC steps of a chunk are unrolled at compile time so every register index is
// static and the scheduler can overlap consecutive steps.
template <typename T, int NC, int RPL, int J, bool WQ, typename TIn>
__device__ __forceinline__ void hh_step(T (&c)[RPL][Slots<NC>::NS], T* Rs, T* red, int q, int p,
                                        int kcol, int spare, Prefetch<T, RPL, TIn>& pf, const VSink<T>& vs)
{
    constexpr int NS = Slots<NC>::NS;
    constexpr int QJ = J % 4, SJ = J / 4;     // lane row and slot holding column J
    constexpr int K = NC - 1 - J;             // trailing columns
    constexpr int OFF = Tri<NC>::off(J);

    // R(J, J) and, for the lane that completes column k, R(J, k): row J of R
    // last changed at step J of the previous chunk, so both reads are issued
    // first and are long complete when needed.  Lanes that own no trailing
    // column read and later write a spare LDS cell, keeping the step free of
    // branches.
    const int k = kcol;
    const bool own = (k > J) && (k < NC);
    const int ridx = own ? OFF + k - J : spare;
    const T alpha = Rs[OFF];
    const T rjk = Rs[ridx];

    // (a) the pivot column in every lane row
    const int src = ((QJ << 4) | p) << 2;
    T x[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) x[r] = bpermute(src, c[r][SJ]);

    // (b) partial dot products of the live slots (slot SJ is live only in
    // lane rows q > QJ; elsewhere its result is ignored), one 16 x 17 LDS tile
    // per lane row: writer p puts slot s at [s][p].  They are issued before
    // the reflector so that its dependent chain runs under the LDS round trip.
    T* rq = red + q * 16 * kRedStride;
    if constexpr (K > 0) {
        static_for<SJ, NS>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            T acc = x[0] * c[0][s];
#pragma unroll
            for (int r = 1; r < RPL; ++r) acc = fmadd(x[r], c[r][s], acc);
            rq[s * kRedStride + p] = acc;
        });
    }
    lds_order();
    // (c) lane (q, p) gathers the 16 partials of column k = 4p + q
    T u[16];
    T fown = T(0);
    if constexpr (K > 0) {
        const T* rd = rq + p * kRedStride;
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = rd[i];
    }

    // the norm of the pivot column and its reflector
    T sp = x[0] * x[0];
#pragma unroll
    for (int r = 1; r < RPL; ++r) sp = fmadd(x[r], x[r], sp);
    const T sigma2 = row_allreduce16(sp);
    const Reflector<T> h = make_reflector(alpha, sigma2);
    if constexpr (WQ) {
        if (q == 0 && J < vs.n) {
            T* col = vs.V + vs.cbase + p + (int64_t)J * vs.ldv;
#pragma unroll
            for (int r = 0; r < RPL; ++r) col[16 * r] = h.s * x[r];
        }
        if (q == 0 && p == 0) vs.tau[J] = h.tau;
    }

    if constexpr (K > 0) {
#pragma unroll
        for (int hh = 8; hh >= 1; hh >>= 1)
#pragma unroll
            for (int i = 0; i < hh; ++i) u[i] = u[i] + u[i + hh];
        const T w = fmadd(h.s, u[0], rjk);
        Rs[ridx] = fmadd(-h.tau, w, rjk);
        fown = own ? h.ts * w : T(0);
    }
    if (q == 0 && p == 0) Rs[OFF] = h.beta;
    lds_order();

    if constexpr (K > 0) {
        // (d) rank-1 update of the live slots; the coefficient of slot s (column
        // 4s + q) is held by lane s of the lane row and reaches the other 15
        // lanes by a row broadcast (DPP row_newbcast), not through LDS
        static_for<SJ, NS>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const T f = dpp_mov<0x150 + s>(fown);
#pragma unroll
            for (int r = 0; r < RPL; ++r) c[r][s] = fmadd(-f, x[r], c[r][s]);
        });
    }

    // (e) slot SJ is finished in every lane row once its last column is the
    // pivot: it takes the next chunk's columns
    if constexpr (QJ == 3 || J == NC - 1) prefetch_slot<T, RPL, NS, TIn>(c, SJ, pf, p);
}

template <typename T, int NC, int RPL, bool WQ, typename TIn>
__device__ __forceinline__ void merge_chunk(T (&c)[RPL][Slots<NC>::NS], T* Rs, T* red, int q, int p,
                                            Prefetch<T, RPL, TIn>& pf, const VSink<T>& vs)
{
    // the column a lane completes in the reduction, passed through an opaque
    // copy so the compiler does not precompute (and keep live) one
    // ownership predicate per step
    int kcol = 4 * p + q;
    asm volatile("" : "+v"(kcol));
    const int spare = Tri<NC>::kSize;      // one LDS cell past the triangle
    static_for<0, NC>([&](auto jc) {
        hh_step<T, NC, RPL, decltype(jc)::value, WQ, TIn>(c, Rs, red, q, p, kcol, spare, pf, vs);
    });
}

// ---- the operator with one column per lane -------------------------------------
//
// R := qr([R1; R2]) for two NC x NC upper triangles, the operator of section 2
// in the structured form of Table 3 (only rows 0..J of R2 take part in step J).
// R1 is packed by rows in LDS (Rs, padded past the triangle); lane k holds
// column k of R2 in registers (v[i] = R2(i, k), zero below the diagonal).  In
// step J every lane fetches the pivot column R2(0:J, J) from lane J's
// registers (ds_bpermute) and forms its own dot product with it locally
// (lane J's is sigma^2, which all lanes then read from its register), so a
// step has no cross-lane reduction, and lane k > J updates R1(J, k) and its
// column.  Used by the reduction tree and the operator entry point,
// where the operands have only NC rows and the length of the dependent chain
// of NC steps, not the arithmetic, sets the time.
//
// Mode::Operator also leaves the Householder vectors in v (lane J's column
// becomes s x, or stays x for an identity reflector) and the tau in tau_out.
enum class Mode { Merge, Operator };

template <typename T, int NC, Mode M>
__device__ __forceinline__ void merge_columns(T (&v)[NC], T* Rs, T* tau_out)
{
    const int lane = lane_id();
    static_for<0, NC>([&](auto jc) {
        constexpr int J = decltype(jc)::value;
        constexpr int OFF = Tri<NC>::off(J);
        const bool own = (lane > J) && (lane < NC);
        const int ridx = own ? OFF + lane - J : Tri<NC>::kSize;
        const T alpha = Rs[OFF];
        const T rjk = Rs[ridx];
        // every lane writes one cell of row J of R1: R1(J, k) for k > J, beta
        // for k = J (no branch), a spare cell otherwise
        const int ridx2 = own ? ridx : ((lane == J) ? OFF : Tri<NC>::kSize);
        // the pivot column, from lane J's registers to every lane
        T x[J + 1];
#pragma unroll
        for (int i = 0; i <= J; ++i) x[i] = bpermute(J << 2, v[i]);
        // this lane's dot product with the pivot column; for lane J it is
        // sigma^2 itself
        // (four partial sums keep the dependent chain short)
        T dd[4] = {x[0] * v[0], T(0), T(0), T(0)};
#pragma unroll
        for (int i = 1; i <= J; ++i) dd[i & 3] = fmadd(x[i], v[i], dd[i & 3]);
        const T d = (dd[0] + dd[1]) + (dd[2] + dd[3]);
        const Reflector<T> h = make_reflector(alpha, lane_value(d, J));
        const T w = fmadd(h.s, d, rjk);
        Rs[ridx2] = own ? fmadd(-h.tau, w, rjk) : ((lane == J) ? h.beta : rjk);
        const T f = own ? h.ts * w : T(0);
#pragma unroll
        for (int i = 0; i <= J; ++i) v[i] = fmadd(-f, x[i], v[i]);
        if constexpr (M == Mode::Operator) {
            const bool mine = (lane == J) && (h.tau != T(0));
#pragma unroll
            for (int i = 0; i <= J; ++i) v[i] = mine ? h.s * x[i] : v[i];
            if (lane == 0) tau_out[J] = h.tau;
        }
        lds_order();
    });
}

// Column `lane` of a packed NC x NC upper triangle held in LDS (rows packed,
// buffer padded to Tri<NC>::kPadded elements so every lane's reads stay inside
// it) into registers, zero below the diagonal and past column NC.
template <typename T, int NC>
__device__ __forceinline__ void triangle_column(const T* tri, T (&v)[NC])
{
    const int k = lane_id();
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const T t = tri[k + (Tri<NC>::off(i) - i)];
        v[i] = (i <= k && k < NC) ? t : T(0);
    }
}

// Copy a packed triangle from global memory to LDS: all loads first, then
// all stores, so the loads are in flight together.
template <typename T, int NC>
__device__ __forceinline__ void triangle_to_lds(const T* __restrict__ src, T* dst)
{
    constexpr int NT = Tri<NC>::kSize;
    constexpr int U = (NT + kWave - 1) / kWave;
    const int lane = lane_id();
    T t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = lane + u * kWave;
        t[u] = src[i < NT ? i : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = lane + u * kWave;
        if (i < NT) dst[i] = t[u];
    }
}

// ---- the fused leaf + tree kernel --------------------------------------------

// One leaf of one instance, then that instance's reduction tree: the body
// shared by the single-matrix kernel and the batched kernel.  `a` describes the
// instance (its matrix, leaf size and count, triangle slots, tree counters and
// output); `leaf` is this workgroup's leaf.  With WQ (the Q-factor mode) the
// leaf also writes its reflectors (a.qs.V, a.qs.tau_leaf), every merge those
// of the operator (a.qs.Vn, a.qs.tau_node), and the root the sign pattern of
// R's diagonal as the starting block of Q (a.qs.qblk, slot 0).  With
// a.stamps set, lane 0 writes the constant-rate clock at the start, at the
// end of the leaf phase and at exit, and the tree level at which it stopped
// (plus 100 for the root), to a.stamps[4 leaf + 0..3]: the split of the time
// between the leaves and the tree, measured.
template <typename T, int NC, int RPL, bool WQ = false, typename TIn = T>
__device__ __forceinline__ void leaf_phase(const LeafTreeArgs<T, TIn>& a, int leaf, T* Rs, T* red)
{
    constexpr int CH = 16 * RPL;                  // rows per chunk
    constexpr int NT = Tri<NC>::kSize;
    constexpr int NS = Slots<NC>::NS;
    const int lane = lane_id();
    const int q = lane >> 4, p = lane & 15;
    const int64_t r0 = (int64_t)leaf * a.leaf_rows;
    const int64_t r1 = (r0 + a.leaf_rows < a.m) ? r0 + a.leaf_rows : a.m;
    const uint64_t t_start = a.stamps ? (uint64_t)wall_clock64() : 0;

    for (int i = lane; i < NT; i += kWave) Rs[i] = T(0);

    // step 1 of the method: the local factorisation of rows [r0, r1)
    if (r1 > r0) {
        T c[RPL][NS];
        {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t row = r0 + p + 16 * r;
                const bool ok = row < r1;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int k = 4 * s + q;
                    c[r][s] = (ok && k < a.n) ? (T)a.A[row + (int64_t)k * a.lda] : T(0);
                }
            }
        }
        wave_sync();
        const int64_t nchunks = (r1 - r0 + CH - 1) / CH;
        for (int64_t t = 0; t < nchunks; ++t) {
            Prefetch<T, RPL, TIn> pf = make_prefetch<T, RPL, TIn>(a.A, a.lda, a.n, r0 + (t + 1) * CH, r1, q, p);
            VSink<T> vs{};
            if constexpr (WQ) {
                vs.V = a.qs.V;
                vs.ldv = a.qs.ldv;
                vs.cbase = r0 + t * CH;
                vs.n = a.n;
                vs.tau = a.qs.tau_leaf + (vs.cbase / CH) * NC;
            }
            merge_chunk<T, NC, RPL, WQ, TIn>(c, Rs, red, q, p, pf, vs);
        }
    }
    wave_sync();
    if (a.stamps && lane == 0) {
        a.stamps[4 * leaf] = t_start;
        a.stamps[4 * leaf + 1] = (uint64_t)wall_clock64();
    }
}

// Step 2 from (node0, level0) on: the triangle of node node0 at tree level
// level0 is in Rs (this wavefront's leaf `leaf`, or the merge of the leaves
// below it); publish it, take the tickets up the tree, merge whenever this
// wavefront arrives second, and finish the root.
template <typename T, int NC, bool WQ = false, typename TIn = T>
__device__ __forceinline__ void tree_phase(const LeafTreeArgs<T, TIn>& a, int leaf, int node0, int level0, T* Rs,
                                           T* red)
{
    constexpr int NT = Tri<NC>::kSize;
    const int lane = lane_id();
    // step 2: binary reduction tree across leaves
    const int P = a.leaves;
    int node = node0;
    int level = level0;
    bool root = ((1 << level) >= P);
    if (!root) {
        T* slot = a.tri + (int64_t)node * NT;
        for (int i = lane; i < NT; i += kWave) slot[i] = Rs[i];
    }
    while (!root) {
        const int span = 1 << level;
        const bool is_left = (node & (2 * span - 1)) == 0;
        const int partner = is_left ? node + span : node - span;
        if (is_left && partner >= P) {          // no partner at this level: carry up
            ++level;
            root = (span * 2 >= P);
            continue;
        }
        const int left = is_left ? node : partner;
        const int id = left + span - 1;         // distinct for every (level, left) pair
        __threadfence();
        unsigned old = 0;
        if (lane == 0) old = atomicAdd(&a.tickets[id], 1u);
        old = (unsigned)__builtin_amdgcn_readfirstlane((int)old);
        if (old == 0) {                         // the partner will merge
            if (a.stamps && lane == 0) {
                a.stamps[4 * leaf + 2] = (uint64_t)wall_clock64();
                a.stamps[4 * leaf + 3] = (uint64_t)level;
            }
            return;
        }
        __threadfence();
        if (lane == 0) a.tickets[id] = 0u;      // both arrived: reset for the next call

        T v[NC];
        if (is_left) {
            triangle_to_lds<T, NC>(a.tri + (int64_t)partner * NT, red);
            wave_sync();
            triangle_column<T, NC>(red, v);
        } else {
            // this wavefront holds the right (lower) operand: move it to registers
            // and bring the left one into LDS, keeping the lower index on top
            triangle_column<T, NC>(Rs, v);
            wave_sync();
            triangle_to_lds<T, NC>(a.tri + (int64_t)partner * NT, Rs);
        }
        wave_sync();
        if constexpr (WQ) {
            // the operator's reflectors: V (the R2 parts, column `lane` in v)
            // and tau (written to LDS by the merge)
            merge_columns<T, NC, Mode::Operator>(v, Rs, red);
            wave_sync();
            T* vn = a.qs.Vn + (int64_t)id * NT;
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (i <= lane && lane < NC) vn[Tri<NC>::off(i) + lane - i] = v[i];
            if (lane < NC) a.qs.tau_node[(int64_t)id * NC + lane] = red[lane];
        } else {
            merge_columns<T, NC, Mode::Merge>(v, Rs, nullptr);
        }
        wave_sync();
        node = left;
        ++level;
        root = ((1 << level) >= P);
        if (!root) {
            T* slot = a.tri + (int64_t)node * NT;
            for (int i = lane; i < NT; i += kWave) slot[i] = Rs[i];
        }
    }

    // root: positive diagonal, +0 below it, leading n-by-n block only
    const int n = a.n;
    for (int idx = lane; idx < n * n; idx += kWave) {
        const int i = idx % n, k = idx / n;
        T v = T(0);
        if (k >= i) {
            v = Rs[Tri<NC>::off(i) + (k - i)];
            if (__builtin_signbit(Rs[Tri<NC>::off(i)])) v = -v;
        }
        a.R[i + (int64_t)k * a.ldr] = v;
    }
    if (a.stamps && lane == 0) {
        a.stamps[4 * leaf + 2] = (uint64_t)wall_clock64();
        a.stamps[4 * leaf + 3] = (uint64_t)(100 + level);
    }
    if constexpr (WQ) {
        // R = D R_raw with D the diagonal of signs, so Q = Q_raw D: the tree
        // pass starts from [D; 0] (identity past column n)
        for (int idx = lane; idx < NC * NC; idx += kWave) {
            const int i = idx % NC, k = idx / NC;
            T d = T(0);
            if (i == k) d = (k < n && __builtin_signbit(Rs[Tri<NC>::off(k)])) ? T(-1) : T(1);
            a.qs.qblk[idx] = d;
        }
    }
}

template <typename T, int NC, int RPL, bool WQ = false, typename TIn = T>
__device__ __forceinline__ void leaf_tree_body(const LeafTreeArgs<T, TIn>& a, int leaf, T* Rs, T* red)
{
    leaf_phase<T, NC, RPL, WQ, TIn>(a, leaf, Rs, red);
    tree_phase<T, NC, WQ, TIn>(a, leaf, leaf, 0, Rs, red);
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup g to XCD g mod 8),
// and each XCD has its own L2.  With P = 8a + b leaves, XCD x runs a + [x < b]
// workgroups; giving them the consecutive leaves starting at x a + min(x, b)
// makes tree siblings share an XCD at every level below the top three, so the
// stores, counters and loads of those merges stay in one L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_local_leaf(int g, int P)
{
    const int a = P / kXcds, b = P % kXcds, x = g % kXcds;
    return x * a + (x < b ? x : b) + g / kXcds;
}

template <typename T, int NC, int RPL, bool WQ = false>
__global__ void __launch_bounds__(kWave) tsqr_leaf_tree_kernel(LeafTreeArgs<T> a)
{
    __shared__ T Rs[Tri<NC>::kPadded];
    __shared__ T red[LdsScratch<NC>::kElems];
    leaf_tree_body<T, NC, RPL, WQ>(a, xcd_local_leaf(blockIdx.x, a.leaves), Rs, red);
}

// Four leaves per workgroup, one wavefront each (one per SIMD of a compute
// unit at one wavefront per SIMD): the two lowest tree levels, whose partners
// then sit in the same workgroup, meet in LDS behind a workgroup barrier
// instead of through global memory, a release fence and a ticket.  Measured
// on a 1024-leaf tree, that global handoff costs 26 us at level 0 and 14 us at
// level 1, where every wavefront fences at once, against 2-6 us above.  The
// merges take the same operands in the same order (the lower index on top),
// so R is bit-identical to tsqr_leaf_tree_kernel's.  P must be a multiple of
// 4; groups are numbered XCD-locally as single leaves are.
template <typename T, int NC, int RPL>
__global__ void __launch_bounds__(4 * kWave) tsqr_leaf_tree4_kernel(LeafTreeArgs<T> a)
{
    __shared__ T Rs[4][Tri<NC>::kPadded];
    __shared__ T red[4][LdsScratch<NC>::kElems];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));   // uniform per wavefront
    const int base = 4 * xcd_local_leaf(blockIdx.x, a.leaves / 4);
    const int leaf = base + w;
    leaf_phase<T, NC, RPL>(a, leaf, Rs[w], red[w]);
    __syncthreads();
    // level 0: leaf base + w (w even) takes base + w + 1 from below
    if ((w & 1) == 0) {
        T v[NC];
        triangle_column<T, NC>(Rs[w + 1], v);
        wave_sync();
        merge_columns<T, NC, Mode::Merge>(v, Rs[w], nullptr);
        wave_sync();
    } else if (a.stamps && lane_id() == 0) {
        a.stamps[4 * leaf + 2] = (uint64_t)wall_clock64();
        a.stamps[4 * leaf + 3] = 0;
    }
    __syncthreads();
    // level 1: base takes base + 2, then the tree goes on through memory
    if (w == 0) {
        T v[NC];
        triangle_column<T, NC>(Rs[2], v);
        wave_sync();
        merge_columns<T, NC, Mode::Merge>(v, Rs[0], nullptr);
        wave_sync();
        tree_phase<T, NC>(a, leaf, base, 2, Rs[0], red[0]);
    } else if (w == 2 && a.stamps && lane_id() == 0) {
        a.stamps[4 * leaf + 2] = (uint64_t)wall_clock64();
        a.stamps[4 * leaf + 3] = 1;
    }
}

// Many independent instances in one launch: workgroup g takes tile
// tiles[g] = (instance, leaf); the tiles are ordered longest first so the
// hardware dispatcher starts the long leaves early and the short ones fill
// in.  Every instance has its own tree, so the tree of one instance overlaps
// the leaves of the others.
//
// With run_if set, the workgroups of an instance whose entry is 0 exit at once
// (the mixed-precision fallback: only instances whose correction failed are
// refactored, decided on the device).  With stamps set, workgroup g writes
// the constant-rate clock when it starts and when it is done (its leaf and
// whatever merges it performed) to stamps[2g], stamps[2g + 1], which measures
// the schedule.  TIn is the storage type of A.
template <typename T, int NC, int RPL, typename TIn = T>
__global__ void __launch_bounds__(kWave) tsqr_batch_kernel(BatchArgs<T, TIn> b)
{
    __shared__ T Rs[Tri<NC>::kPadded];
    __shared__ T red[LdsScratch<NC>::kElems];
    const uint64_t t_start = b.stamps ? (uint64_t)wall_clock64() : 0;
    const BatchTile t = b.tiles[blockIdx.x];
    if (b.run_if && b.run_if[t.inst] == 0) return;
    const BatchInstance in = b.inst[t.inst];
    LeafTreeArgs<T, TIn> a;
    a.A = b.A + in.a_off;
    a.m = in.m;
    a.lda = in.lda;
    a.n = b.n;
    a.leaf_rows = in.leaf_rows;
    a.leaves = in.leaves;
    a.tri = b.tri + in.tri_off;
    a.tickets = b.tickets + in.ticket_off;
    a.R = b.R + (int64_t)t.inst * b.ldr * b.n;
    a.ldr = b.ldr;
    a.qs = QStore<T>{};
    leaf_tree_body<T, NC, RPL, false, TIn>(a, t.leaf, Rs, red);
    if (b.stamps && threadIdx.x == 0) {
        b.stamps[2 * blockIdx.x] = t_start;
        b.stamps[2 * blockIdx.x + 1] = (uint64_t)wall_clock64();
    }
}

// ---- the paper's operator as a single-workgroup kernel -------------------------

template <typename T, int NC>
__global__ void __launch_bounds__(kWave) qr_uppers_kernel(int n, T* R1, T* R2, T* tau)
{
    constexpr int NT = Tri<NC>::kSize;
    __shared__ T Rs[Tri<NC>::kPadded];
    __shared__ T R2s[Tri<NC>::kPadded];
    __shared__ T taus[NC];
    const int lane = threadIdx.x;
    for (int idx = lane; idx < NT; idx += kWave) {
        // packed index -> (row, column)
        int i = 0;
        while (Tri<NC>::off(i + 1) <= idx) ++i;
        const int k = i + (idx - Tri<NC>::off(i));
        const bool in = i < n && k < n;
        Rs[idx] = in ? R1[i + (int64_t)k * n] : T(0);
        R2s[idx] = in ? R2[i + (int64_t)k * n] : T(0);
    }
    wave_sync();
    T v[NC];
    triangle_column<T, NC>(R2s, v);
    wave_sync();
    merge_columns<T, NC, Mode::Operator>(v, Rs, taus);
    wave_sync();
    for (int idx = lane; idx < n * n; idx += kWave) {
        const int i = idx % n, k = idx / n;
        if (k >= i) R1[idx] = Rs[Tri<NC>::off(i) + (k - i)];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i)
        if (i <= lane && lane < n) R2[i + (int64_t)lane * n] = v[i];
    if (lane < n) tau[lane] = taus[lane];
}

}  // namespace dev
}  // namespace tsqr
