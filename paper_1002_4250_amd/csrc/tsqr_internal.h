// tsqr_internal.h -- declarations shared by the C-ABI layer and the kernel
// instantiation units of libtsqr.so (the public interface is include/tsqr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsqr_instances.h"

namespace tsqr {

template <typename T>
struct LeafTreeArgs {
    const T* A;           // m-by-n, column-major
    int64_t m;
    int64_t lda;
    int n;
    int64_t leaf_rows;    // rows per leaf (multiple of the chunk)
    int leaves;           // P = ceil(m / leaf_rows), at least 1
    T* tri;               // workspace: P packed triangles
    unsigned* tickets;    // workspace: P tree counters, zero on entry and on exit
    T* R;                 // n-by-n output
    int64_t ldr;
};

using f64 = double;
using f32 = float;

#define TSQR_DECLARE_LEAF(tag, NC, RPL) \
    hipError_t launch_leaf_tree_##tag##_##NC##_##RPL(const LeafTreeArgs<tag>& a, hipStream_t s);
#define TSQR_DECLARE_OP(tag, NC) \
    hipError_t launch_qr_uppers_##tag##_##NC(int n, tag* R1, tag* R2, tag* tau, hipStream_t s);
TSQR_LEAF_INSTANCES(TSQR_DECLARE_LEAF)
TSQR_OP_INSTANCES(TSQR_DECLARE_OP)
#undef TSQR_DECLARE_LEAF
#undef TSQR_DECLARE_OP

hipError_t launch_zero_u32(unsigned* p, int64_t count, hipStream_t s);

}  // namespace tsqr
