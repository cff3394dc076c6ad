// tsqr_device.h -- gfx950 device code for the R factor of a tall-skinny matrix
// by Householder TSQR (Langou, arXiv:1002.4250, sections 2-3).
//
// Execution model (one wavefront of 64 lanes per workgroup):
//   * A leaf is a contiguous block of rows of A.  Its wavefront keeps the n-by-n
//     triangle R in LDS (packed by rows) and streams the block through
//     registers in chunks of 64*RPL rows; chunk rows are distributed one per
//     lane per register slot (lane l holds rows base + l + 64*r, r < RPL, all
//     NC columns).  Each chunk C is merged into R by R := R-factor of [R; C]:
//     for every column j one Householder reflector built from R(j,j) and
//     C(:,j) is applied to the trailing columns (the structured update of
//     Table 3 with R2 replaced by a dense chunk: a flat tree inside the leaf,
//     section 2 allows any tree).
//   * Leaves then combine with the paper's operator qr(R1, R2) over a binary
//     tree pairing leaf i with i + 2^level (lower index on top), the merge done
//     by whichever wavefront of the pair arrives last (atomic ticket), so no
//     wavefront ever waits on another.
//   * The root flips rows with a negative diagonal (section 2's positive
//     diagonal convention) and writes R.
//
// Per Householder step j (K = NC-1-j trailing columns, x = C(:,j)):
//     d_0 = x.x, d_v = x.C(:,j+v)                 (partials in registers, then a
//                                                  64-lane transpose-reduction)
//     beta = -sign(alpha) sqrt(alpha^2 + d_0), alpha = R(j,j)
//     tau = (beta - alpha)/beta, s = 1/(alpha - beta)        (v = s x)
//     w_v = R(j,j+v) + s d_v,  R(j,j+v) -= tau w_v,  C(:,j+v) -= (tau s w_v) x
// which is the reflector generation and rank-1 update of Table 3 with the
// Householder vector kept unscaled (v = s x) so that no lane has to rescale
// its rows before the dot products.
//
// The transpose-reduction of V = K+1 values uses the gfx950 lane-swap
// instructions: v_permlane32_swap pairs values (2q, 2q+1) across the two
// 32-lane halves, v_permlane16_swap pairs the results across 16-lane rows,
// and the last 16-to-1 sum goes through LDS, after which lane 16*r + p holds
// the full sum of value 4p + 2(r&1) + (r>>1).
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
constexpr int kRedElems = 4 * 16 * kRedStride;
#ifndef TSQR_GROUP
#define TSQR_GROUP 8
#endif
constexpr int kGroup = TSQR_GROUP;              // update coefficients read per group

template <int NC>
struct Tri {
    static constexpr int kSize = NC * (NC + 1) / 2;
    // packed row-major upper triangle: row j starts at off(j), entry (j,k) at off(j)+k-j
    static constexpr __host__ __device__ int off(int j) { return j * NC - (j * (j - 1)) / 2; }
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

// Lanes 0-31 return a(l) + a(l+32); lanes 32-63 return b(l-32) + b(l).
__device__ __forceinline__ double pair32(double a, double b)
{
    unsigned alo = (unsigned)__double2loint(a), ahi = (unsigned)__double2hiint(a);
    unsigned blo = (unsigned)__double2loint(b), bhi = (unsigned)__double2hiint(b);
    auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float pair32(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// Within each pair of 16-lane rows (0,1) and (2,3): even rows return a summed
// over the two rows, odd rows return b summed over the two rows.
__device__ __forceinline__ double pair16(double a, double b)
{
    unsigned alo = (unsigned)__double2loint(a), ahi = (unsigned)__double2hiint(a);
    unsigned blo = (unsigned)__double2loint(b), bhi = (unsigned)__double2hiint(b);
    auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float pair16(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ double readlane(double x, int l)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// Lane that holds reduced value v after transpose_reduce.
__host__ __device__ constexpr int holder_lane(int v)
{
    return 16 * (((v & 1) << 1) | ((v >> 1) & 1)) + (v >> 2);
}

// ---- one Householder step ----------------------------------------------------

enum class Mode { Leaf, Merge, Operator };

// Where a leaf prefetches its next chunk from: a running pointer to column J
// of the next chunk, advanced by lda after every step.  lda and the column
// count pass through an opaque register copy at every chunk so that the
// compiler keeps one running pointer instead of precomputing (and keeping
// live) one address and one predicate per column.
template <typename T, int RPL>
struct Prefetch {
    const T* col;        // uniform: &A(base, J)
    int64_t lda;         // uniform
    int cols_left;       // uniform: columns J..n-1 still to load
    bool ok[RPL];        // per lane: row base + lane + 64 r lies inside the leaf
};

template <typename T, int RPL>
__device__ __forceinline__ Prefetch<T, RPL> make_prefetch(const T* A, int64_t lda, int n, int64_t base, int64_t r1,
                                                          int lane)
{
    Prefetch<T, RPL> pf;
    int64_t ld = lda;
    int nn = n;
    asm volatile("" : "+s"(ld), "+s"(nn));
    pf.col = A + (base < r1 ? base : 0);
    pf.lda = ld;
    pf.cols_left = nn;
#pragma unroll
    for (int r = 0; r < RPL; ++r) pf.ok[r] = base + lane + kWave * r < r1;
    return pf;
}

template <typename T, int NC, int RPL>
__device__ __forceinline__ void prefetch_column(T (&c)[RPL][NC], int J, Prefetch<T, RPL>& pf, int lane)
{
    if (pf.cols_left > 0) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) c[r][J] = pf.ok[r] ? pf.col[lane + kWave * r] : T(0);
    } else {
#pragma unroll
        for (int r = 0; r < RPL; ++r) c[r][J] = T(0);
    }
    pf.col += pf.lda;
    pf.cols_left -= 1;
}

// Step J of R := qr([R; C]) with R packed in LDS (Rs) and C in registers.
template <typename T, int NC, int RPL, Mode M, int J>
__device__ __forceinline__ void hh_step(T (&c)[RPL][NC], T* Rs, T* red, T* F, int lane,
                                        Prefetch<T, RPL>& pf, T* tau_out)
{
    constexpr int K = NC - 1 - J;
    constexpr int V = K + 1;
    constexpr int HA = (V + 1) / 2;
    constexpr int HB = (HA + 1) / 2;
    constexpr int OFF = Tri<NC>::off(J);

    auto dot = [&](auto vc) -> T {
        constexpr int v = decltype(vc)::value;
        if constexpr (v >= V) {
            return T(0);
        } else {
            T s = c[0][J] * c[0][J + v];
#pragma unroll
            for (int r = 1; r < RPL; ++r) s = __builtin_fma(c[r][J], c[r][J + v], s);
            return s;
        }
    };

    // stages A and B, fused with the production of the partial dot products
    T b[HB];
    static_for<0, HB>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        T a0 = pair32(dot(std::integral_constant<int, 4 * t>{}), dot(std::integral_constant<int, 4 * t + 1>{}));
        T a1 = pair32(dot(std::integral_constant<int, 4 * t + 2>{}), dot(std::integral_constant<int, 4 * t + 3>{}));
        b[t] = pair16(a0, a1);
    });

    // stage C: 16-to-1 through LDS (writer-major rows, odd stride)
    const int row = lane >> 4, pos = lane & 15;
    T* rb = red + row * 16 * kRedStride;
#pragma unroll
    for (int t = 0; t < HB; ++t) rb[pos * kRedStride + t] = b[t];
    wave_sync();
    T u[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = rb[i * kRedStride + pos];
#pragma unroll
    for (int h = 8; h >= 1; h >>= 1)
#pragma unroll
        for (int i = 0; i < h; ++i) u[i] = u[i] + u[i + h];
    const T d = u[0];
    const int vh = 4 * pos + 2 * (row & 1) + (row >> 1);   // value index held by this lane

    // reflector (uniform across the wave)
    const T sigma2 = readlane(d, 0);
    const T alpha = Rs[OFF];
    T tau = T(0), s = T(0), beta = alpha;
    if (sigma2 >= Limits<T>::tiny) {
        const T nrm = __builtin_sqrt(__builtin_fma(alpha, alpha, sigma2));
        beta = __builtin_signbit(alpha) ? nrm : -nrm;
        tau = (beta - alpha) / beta;
        s = T(1) / (alpha - beta);
    }
    const T ts = tau * s;

    if constexpr (K > 0) {
        if (vh >= 1 && vh <= K) {
            const T rjk = Rs[OFF + vh];
            const T w = __builtin_fma(s, d, rjk);
            Rs[OFF + vh] = __builtin_fma(-tau, w, rjk);
            F[vh - 1] = ts * w;
        }
    }
    if (lane == 0) Rs[OFF] = beta;
    wave_sync();
    if constexpr (K > 0) {
        // rank-1 update, reading the K coefficients in groups of kGroup so that
        // at most two groups are live in registers (reads of group g+1 overlap
        // the FMAs of group g)
        constexpr int NG = (K + kGroup - 1) / kGroup;
        T f[2][kGroup];
        auto load_group = [&](auto gc, T (&dst)[kGroup]) {
            constexpr int g = decltype(gc)::value;
#pragma unroll
            for (int i = 0; i < kGroup; ++i)
                if (g * kGroup + i < K) dst[i] = F[g * kGroup + i];
        };
        load_group(std::integral_constant<int, 0>{}, f[0]);
        static_for<0, NG>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            if constexpr (g + 1 < NG) load_group(std::integral_constant<int, g + 1>{}, f[(g + 1) & 1]);
#pragma unroll
            for (int i = 0; i < kGroup; ++i) {
                const int v = 1 + g * kGroup + i;
                if (v <= K) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r)
                        c[r][J + v] = __builtin_fma(-f[g & 1][i], c[r][J], c[r][J + v]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    if constexpr (M == Mode::Operator) {
        // the Householder vector v = s x replaces x (identity reflector: x kept)
        if (tau != T(0)) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) c[r][J] = s * c[r][J];
        }
        if (lane == 0) tau_out[J] = tau;
    } else if constexpr (M == Mode::Leaf) {
        // column J of this chunk is finished: its registers take the next chunk's column J
        prefetch_column<T, NC, RPL>(c, J, pf, lane);
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <typename T, int NC, int RPL, Mode M>
__device__ __forceinline__ void merge_chunk(T (&c)[RPL][NC], T* Rs, T* red, T* F, int lane,
                                            Prefetch<T, RPL>& pf, T* tau_out)
{
    static_for<0, NC>([&](auto jc) {
        hh_step<T, NC, RPL, M, decltype(jc)::value>(c, Rs, red, F, lane, pf, tau_out);
    });
}

// Load the packed triangle `tri` (NC*(NC+1)/2 values, rows packed; LDS or
// global) into registers one row per lane: lane i holds R(i, k) for k >= i,
// zero elsewhere.
template <typename T, int NC>
__device__ __forceinline__ void triangle_to_rows(const T* tri, T (&c)[1][NC], int lane)
{
    const int base = (lane < NC) ? Tri<NC>::off(lane) - lane : 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) c[0][k] = (lane < NC && k >= lane) ? tri[base + k] : T(0);
}

// ---- the fused leaf + tree kernel --------------------------------------------

template <typename T, int NC, int RPL>
__global__ void __launch_bounds__(kWave) tsqr_leaf_tree_kernel(LeafTreeArgs<T> p)
{
    constexpr int CH = kWave * RPL;
    constexpr int NT = Tri<NC>::kSize;
    __shared__ T Rs[NT];
    __shared__ T red[kRedElems];
    __shared__ T F[kWave];
    const int lane = threadIdx.x;
    const int leaf = blockIdx.x;
    const int64_t r0 = (int64_t)leaf * p.leaf_rows;
    const int64_t r1 = (r0 + p.leaf_rows < p.m) ? r0 + p.leaf_rows : p.m;

    for (int i = lane; i < NT; i += kWave) Rs[i] = T(0);

    // step 1 of the method: the local factorisation of rows [r0, r1)
    if (r1 > r0) {
        T c[RPL][NC];
        {
            Prefetch<T, RPL> first = make_prefetch<T, RPL>(p.A, p.lda, p.n, r0, r1, lane);
#pragma unroll
            for (int j = 0; j < NC; ++j) prefetch_column<T, NC, RPL>(c, j, first, lane);
        }
        wave_sync();
        const int64_t nchunks = (r1 - r0 + CH - 1) / CH;
        for (int64_t t = 0; t < nchunks; ++t) {
            Prefetch<T, RPL> pf = make_prefetch<T, RPL>(p.A, p.lda, p.n, r0 + (t + 1) * CH, r1, lane);
            merge_chunk<T, NC, RPL, Mode::Leaf>(c, Rs, red, F, lane, pf, nullptr);
        }
    }
    wave_sync();

    // step 2: binary reduction tree across leaves
    const int P = p.leaves;
    int node = leaf;
    int level = 0;
    bool root = (P == 1);
    if (!root) {
        T* slot = p.tri + (int64_t)node * NT;
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
        if (lane == 0) old = atomicAdd(&p.tickets[id], 1u);
        old = (unsigned)__builtin_amdgcn_readfirstlane((int)old);
        if (old == 0) return;                   // the partner will merge
        __threadfence();
        if (lane == 0) p.tickets[id] = 0u;      // both arrived: reset for the next call

        T c1[1][NC];
        if (is_left) {
            triangle_to_rows<T, NC>(p.tri + (int64_t)partner * NT, c1, lane);
        } else {
            // this wavefront holds the right (lower) operand: move it to registers
            // and bring the left one into LDS, keeping the lower index on top
            triangle_to_rows<T, NC>(Rs, c1, lane);
            wave_sync();
            const T* lt = p.tri + (int64_t)partner * NT;
            for (int i = lane; i < NT; i += kWave) Rs[i] = lt[i];
        }
        wave_sync();
        Prefetch<T, 1> none{};
        merge_chunk<T, NC, 1, Mode::Merge>(c1, Rs, red, F, lane, none, nullptr);
        wave_sync();
        node = left;
        ++level;
        root = ((1 << level) >= P);
        if (!root) {
            T* slot = p.tri + (int64_t)node * NT;
            for (int i = lane; i < NT; i += kWave) slot[i] = Rs[i];
        }
    }

    // root: positive diagonal, +0 below it, leading n-by-n block only
    const int n = p.n;
    for (int idx = lane; idx < n * n; idx += kWave) {
        const int i = idx % n, k = idx / n;
        T v = T(0);
        if (k >= i) {
            v = Rs[Tri<NC>::off(i) + (k - i)];
            if (__builtin_signbit(Rs[Tri<NC>::off(i)])) v = -v;
        }
        p.R[i + (int64_t)k * p.ldr] = v;
    }
}

// ---- the paper's operator as a single-workgroup kernel -------------------------

template <typename T, int NC>
__global__ void __launch_bounds__(kWave) qr_uppers_kernel(int n, T* R1, T* R2, T* tau)
{
    constexpr int NT = Tri<NC>::kSize;
    __shared__ T Rs[NT];
    __shared__ T red[kRedElems];
    __shared__ T F[kWave];
    __shared__ T taus[NC];
    const int lane = threadIdx.x;
    for (int idx = lane; idx < NT; idx += kWave) {
        // packed index -> (row, column)
        int i = 0;
        while (Tri<NC>::off(i + 1) <= idx) ++i;
        const int k = i + (idx - Tri<NC>::off(i));
        Rs[idx] = (i < n && k < n) ? R1[i + (int64_t)k * n] : T(0);
    }
    T c[1][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) c[0][k] = (lane < n && k < n && k >= lane) ? R2[lane + (int64_t)k * n] : T(0);
    wave_sync();
    Prefetch<T, 1> none{};
    merge_chunk<T, NC, 1, Mode::Operator>(c, Rs, red, F, lane, none, taus);
    wave_sync();
    for (int idx = lane; idx < n * n; idx += kWave) {
        const int i = idx % n, k = idx / n;
        if (k >= i) R1[idx] = Rs[Tri<NC>::off(i) + (k - i)];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (lane < n && k < n && k >= lane) R2[lane + (int64_t)k * n] = c[0][k];
    if (lane < n) tau[lane] = taus[lane];
}

}  // namespace dev
}  // namespace tsqr
