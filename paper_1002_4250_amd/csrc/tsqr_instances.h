// tsqr_instances.h -- the kernel instantiations compiled into libtsqr.so.
// Each X(tag, NC, RPL) is a leaf+tree kernel for element type tag (f64/f32),
// NC compiled columns and RPL rows per lane (a chunk is 16*RPL rows); each O(tag, NC) an operator
// kernel (with the mixed-precision kernels for f64); each Q(tag, NC, RPL) the Q-factor kernels.  The build compiles one translation unit per entry (in parallel) and
// the C-ABI layer dispatches through the same lists.
#pragma once

#define TSQR_LEAF_INSTANCES(X) \
    X(f64, 16, 8) X(f64, 32, 8) X(f64, 50, 4) X(f64, 50, 6) X(f64, 50, 8) X(f64, 64, 8) \
    X(f32, 16, 8) X(f32, 32, 8) X(f32, 50, 8) X(f32, 50, 12) X(f32, 50, 16) X(f32, 64, 8)

#define TSQR_OP_INSTANCES(O) \
    O(f64, 16) O(f64, 32) O(f64, 50) O(f64, 64) \
    O(f32, 16) O(f32, 32) O(f32, 50) O(f32, 64)

// Q-factor mode: leaf+tree kernel storing reflectors, tree pass, leaf pass
#define TSQR_QR_INSTANCES(Q) \
    Q(f64, 16, 8) Q(f64, 32, 8) Q(f64, 50, 8) Q(f64, 64, 8) \
    Q(f32, 16, 8) Q(f32, 32, 8) Q(f32, 50, 8) Q(f32, 64, 8)

// column counts with a compiled kernel (ascending) and the default rows per lane
#define TSQR_NC_VALUES 16, 32, 50, 64
#define TSQR_DEFAULT_RPL_F64 8
#define TSQR_DEFAULT_RPL_F32 8
