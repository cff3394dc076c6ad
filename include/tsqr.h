/*
 * tsqr.h -- C ABI of libtsqr.so: the R factor of a tall-skinny matrix by
 * Householder TSQR on one AMD MI355X (gfx950) GPU.
 *
 * Method: J. Langou, "Computing the R of the QR factorization of tall and
 * skinny matrices using MPI_Reduce" (arXiv:1002.4250).  The rows of A are split
 * into blocks, each block is reduced to an n-by-n upper triangle by Householder
 * reflections (step 1 of section 2), and the triangles are combined by the
 * associative operator R := qr(R1, R2) of section 2 / Table 3 over a binary
 * reduction tree (step 2; the hand-made binary tree of section 4).  On the GPU
 * a block is the rows one wavefront streams through its on-chip triangle, and
 * the tree runs across workgroups instead of across MPI ranks.
 *
 * Conventions shared by every entry point:
 *  - Matrices are column-major: element (i, j) of a matrix with leading
 *    dimension ld is at index i + j*ld.
 *  - Every pointer to matrix data is a DEVICE pointer owned by the caller
 *    (e.g. from hipMalloc or a PyTorch tensor).  The library never frees,
 *    retains or allocates caller memory, and the compute entry points allocate
 *    nothing: scratch space is the caller's workspace buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Compute calls are asynchronous on that stream; argument checks happen
 *    synchronously on the host before any HIP call.
 *  - Return status: 0 = success; -k = argument k (1-based, handle counted)
 *    is invalid and nothing was launched; positive values are the TSQR_ERR_*
 *    codes below.
 *  - Supported column counts: 1 <= n <= TSQR_MAX_N (n = 0 is a no-op).
 *  - Output convention (section 2: R is unique up to row signs; fixing the
 *    diagonal sign makes it unique): R has a non-negative diagonal and +0.0
 *    below the diagonal.  Only the leading n-by-n block of R is written.
 *  - Numerical range: column norms are formed as plain sums of squares in the
 *    working precision, so entries must stay within about 1e+-150 (FP64) or
 *    1e+-18 (FP32) of unity; a column whose remaining sum of squares is below
 *    the smallest normal number is treated as exactly zero (identity
 *    reflector).  NaN and Inf propagate; nothing in the hot path checks.
 *  - Results are bit-reproducible from run to run for fixed (m, n, lda,
 *    options): the tree pairing and the operand order of every merge are fixed.
 */
#ifndef TSQR_H
#define TSQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSQR_MAX_N 64

/* element types */
#define TSQR_F64 0
#define TSQR_F32 1

/* positive status codes */
#define TSQR_ERR_HIP 1          /* a HIP runtime call failed: tsqr_last_hip_error() */
#define TSQR_ERR_UNSUPPORTED 2  /* n > TSQR_MAX_N, or a size beyond the kernels' index range */
#define TSQR_ERR_NO_DEVICE 3    /* no usable gfx950 device */
#define TSQR_ERR_ALLOC 4        /* host or device allocation failed (plan creation only) */
#define TSQR_ERR_SCRATCH 5      /* tsqr_geqr_r_f64_noalloc: the problem needs more than its fixed scratch */

/* options for tsqr_set_option (0 restores the automatic choice) */
#define TSQR_OPT_LEAF_ROWS 1      /* rows per leaf block; rounded up to a whole chunk */
#define TSQR_OPT_ROWS_PER_LANE 2  /* rows each lane holds per chunk (chunk = 16 x this rows); only
                                     compiled values take effect, others fall back */
#define TSQR_OPT_WAVES_PER_CU 3   /* leaves per compute unit for the automatic leaf size
                                     (automatic: as many as are resident on a compute unit) */

typedef struct tsqr_handle_s *tsqr_handle_t;
typedef struct tsqr_batch_plan_s *tsqr_batch_plan_t;
typedef struct tsqr_mixed_plan_s *tsqr_mixed_plan_t;

/* Create a handle bound to HIP device `device` (which becomes current on the
 * calling thread).  Reads the device's compute-unit count for the launch
 * policy.  Returns TSQR_ERR_NO_DEVICE if the device does not exist or is not a
 * gfx950.  The handle owns no caller memory. */
int tsqr_create(tsqr_handle_t *handle, int device);

/* Create a planning-only handle that is bound to no device, with `cu_count`
 * compute units assumed for the launch policy (e.g. 256 for an MI355X).  It
 * answers tsqr_workspace_bytes and tsqr_plan_info and runs every argument
 * check; compute calls on it return TSQR_ERR_NO_DEVICE once their arguments
 * have been checked.  Makes no HIP call. */
int tsqr_create_planning(tsqr_handle_t *handle, int cu_count);

/* Destroy a handle (NULL is accepted). */
int tsqr_destroy(tsqr_handle_t handle);

/* The last hipError_t seen by a call on this handle (0 if none). */
int tsqr_last_hip_error(tsqr_handle_t handle);

/* Static description of a status code. */
const char *tsqr_status_string(int status);

/* Set a tuning option (see TSQR_OPT_*).  Negative values are rejected. */
int tsqr_set_option(tsqr_handle_t handle, int option, int64_t value);

/* ---- tuning table ---------------------------------------------------------------
 *
 * The launch configuration that the automatic policy uses can come from a
 * table measured on the device (paper_1002_4250_amd/autotune.py writes one).
 * An entry applies to calls of element type `dtype` whose column count pads to
 * the same compiled width as `n`:
 *   batch == 0: single-matrix calls (tsqr_geqr_r_*, tsqr_plan_info,
 *               tsqr_workspace_bytes, tsqr_geqr_qr_f64) with m <= m_max; of
 *               several such entries the one with the smallest m_max wins;
 *   batch != 0: batched plans (m_max is ignored).
 * It sets the rows per lane (a compiled value for that width; the Q-factor
 * entry point keeps its fixed 8) and the leaf size: `leaf_rows` if positive,
 * else `waves_per_cu` leaves per compute unit if positive, else the built-in
 * policy.  Options set with tsqr_set_option take precedence over the table.
 * An entry with the same key (dtype, width, batch, and m_max for single-matrix
 * entries) replaces the earlier one.  Host-only; changes plans made after the
 * call, not existing batched plans.  Like tsqr_set_option, it must not run
 * concurrently with other calls on the same handle.  Argument codes: -1 handle, -2 dtype,
 * -3 n (not in 1..TSQR_MAX_N), -4 m_max, -5 rows_per_lane (not compiled for
 * this width), -6 waves_per_cu, -7 leaf_rows; TSQR_ERR_UNSUPPORTED once the
 * table holds 4096 entries. */
int tsqr_tuning_add(tsqr_handle_t handle, int dtype, int64_t n, int64_t m_max, int64_t rows_per_lane,
                    int64_t waves_per_cu, int64_t leaf_rows, int batch);
/* Remove every entry of the handle's tuning table. */
int tsqr_tuning_clear(tsqr_handle_t handle);
/* The rows-per-lane values compiled for (dtype, width of n): writes up to
 * `capacity` of them to the host array `values` and returns how many exist;
 * -1 dtype, -2 n, -3 values/capacity. */
int64_t tsqr_rows_per_lane_compiled(int dtype, int64_t n, int64_t *values, int64_t capacity);

/* Launch geometry tsqr_geqr_r_* will use for (m, n, dtype): rows per leaf and
 * number of leaves (workgroups).  Either output pointer may be NULL. */
int tsqr_plan_info(tsqr_handle_t handle, int64_t m, int64_t n, int dtype,
                   int64_t *leaf_rows, int64_t *leaves);

/* Workspace bytes needed by tsqr_geqr_r_* for (m, n, dtype) with the handle's
 * current options (the analogue of LAPACK's lwork = -1 query, Table 1's
 * dgeqrf call).  Returns a negative argument code on bad input, or
 * -1000 - status for an unsupported size.  The workspace holds one tree
 * counter per leaf (at its start) and one packed triangle per leaf. */
int64_t tsqr_workspace_bytes(tsqr_handle_t handle, int64_t m, int64_t n, int dtype);


/* R factor of the m-by-n matrix A (the "two-line code" of Table 1 fused into
 * one call: local Householder QR of every row block, then the reduction of
 * the block triangles with qr_uppers over a binary tree).
 *   A    device, m-by-n, column-major, lda >= max(1, m); read only.
 *   R    device, n-by-n output, column-major, ldr >= max(1, n).
 *   ws   device workspace of at least tsqr_workspace_bytes(...) bytes,
 *        256-byte aligned; contents on entry are irrelevant and are
 *        overwritten; calls that may run concurrently must not share a
 *        workspace.
 * The call makes two kernel launches (a small one that zeroes the tree
 * counters, then the factorisation) and allocates nothing.
 * m = 0 gives R = 0; m < n gives zero rows m..n-1 (the missing rows are
 * read as zeros).  Argument codes: -1 handle, -2 m, -3 n, -4 A, -5 lda, -6 R,
 * -7 ldr, -8 ws, -9 ws_bytes. */
int tsqr_geqr_r_f64(tsqr_handle_t handle, int64_t m, int64_t n, const double *A, int64_t lda,
                    double *R, int64_t ldr, void *ws, int64_t ws_bytes, void *stream);
int tsqr_geqr_r_f32(tsqr_handle_t handle, int64_t m, int64_t n, const float *A, int64_t lda,
                    float *R, int64_t ldr, void *ws, int64_t ws_bytes, void *stream);

/* tsqr_geqr_r_f64 that also measures where the time goes: lane 0 of leaf i's
 * wavefront writes, to stamps[4i .. 4i+3] (device memory owned by the caller,
 * 4 x leaves values, leaves from tsqr_plan_info): the device's constant-rate
 * clock (tsqr_device_clock_khz) when it starts, when its leaf phase (step 1
 * of section 2) is done and when it exits, and the tree level at which it
 * stopped (the first to arrive at a merge stops there), plus 100 for the
 * wavefront that finished the root.  R is
 * bit-identical to tsqr_geqr_r_f64's.  Argument codes as tsqr_geqr_r_f64's,
 * plus -10 stamps. */
int tsqr_geqr_r_f64_stamped(tsqr_handle_t handle, int64_t m, int64_t n, const double *A, int64_t lda, double *R,
                            int64_t ldr, void *ws, int64_t ws_bytes, uint64_t *stamps, void *stream);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): tsqr_geqr_r_f64 with the workspace taken from a fixed array that
 * the library holds on every device it runs on (TSQR_NOALLOC_SCRATCH_BYTES per
 * device, kept until the process ends; its address is looked up once per
 * device when a handle is created).  Same arguments as tsqr_geqr_r_f64 minus
 * the workspace; same kernels, launch geometry and result, bit for bit.  The
 * call allocates nothing: it launches the counter-clearing kernel and the
 * factorization on `stream`.  All calls on one device share the array, so
 * calls that may overlap on one device (other streams, other threads, other
 * handles) race and must be serialized by the caller.  Returns
 * TSQR_ERR_SCRATCH, before any launch, if the workspace the plan needs (see
 * tsqr_workspace_bytes) exceeds TSQR_NOALLOC_SCRATCH_BYTES: with the
 * built-in leaf policy on an MI355X (at most 1024 leaves in FP64, 17 MB at
 * n = 64) every n <= TSQR_MAX_N and any m fit; a small TSQR_OPT_LEAF_ROWS or
 * a large TSQR_OPT_WAVES_PER_CU on a large m can exceed it.  Argument codes: -1
 * handle, -2 m, -3 n, -4 A, -5 lda, -6 R, -7 ldr. */
#define TSQR_NOALLOC_SCRATCH_BYTES ((int64_t)32 << 20)
int tsqr_geqr_r_f64_noalloc(tsqr_handle_t handle, int64_t m, int64_t n, const double *A, int64_t lda,
                            double *R, int64_t ldr, void *stream);

/* The paper's reduction operator (section 3, Table 3: LILA_qr_uppers) on two
 * n-by-n upper triangles stacked as [R1; R2], same contract:
 *   R1   device, n-by-n, leading dimension n; on exit its upper triangle holds
 *        R (diagonal signs as the reflectors leave them: no normalisation).
 *   R2   device, n-by-n, leading dimension n; on exit its upper triangle holds
 *        the Householder vectors V, the reflectors being H_j = I - tau_j
 *        [e_j; V(:,j)] [e_j; V(:,j)]^T.
 *   tau  device, n scalars.
 * Only the upper triangles of R1 and R2 are read or written.  One workgroup
 * computes the operator; the call is latency-bound by design.  Argument
 * codes: -1 handle, -2 n, -3 R1, -4 R2, -5 tau. */
int tsqr_qr_uppers_f64(tsqr_handle_t handle, int64_t n, double *R1, double *R2, double *tau,
                       void *stream);
int tsqr_qr_uppers_f32(tsqr_handle_t handle, int64_t n, float *R1, float *R2, float *tau,
                       void *stream);

/* ---- many independent matrices in one launch ------------------------------
 *
 * A batch of `batch` matrices with the same column count n and individual row
 * counts m[b] (any mix of sizes, e.g. 64 to 65536 rows).  Every instance gets
 * the method of section 2 (local QR of its row blocks, then its own binary
 * tree of qr_uppers merges); the (instance, block) tiles of all instances run
 * in ONE kernel launch, longest blocks first, so the trees of some instances
 * overlap the block factorisations of others.  A plan holds the tile schedule
 * on the device; executing it allocates nothing and is safe to capture in a
 * HIP graph (its two launches are kernels, no memset).
 *
 * Create: m, a_offset, lda are HOST arrays of `batch` entries: instance b is
 * the m[b]-by-n column-major matrix at element offset a_offset[b] of the A
 * pointer given to tsqr_batch_exec, with leading dimension lda[b] (NULL:
 * lda[b] = max(1, m[b])).  The leaf size is the handle's TSQR_OPT_LEAF_ROWS if
 * set, else the tuning table's batched entry, else 64 chunks; rows per lane
 * likewise (option, table, built-in default).  The plan allocates two small device tables (freed by
 * tsqr_batch_plan_destroy) and keeps a pointer to the handle, which must
 * outlive it.  Argument codes: -1 handle, -2 batch, -3 n, -4 m, -5 a_offset,
 * -6 lda, -7 dtype, -8 plan. */
int tsqr_batch_plan_create(tsqr_handle_t handle, int64_t batch, int64_t n, const int64_t *m,
                           const int64_t *a_offset, const int64_t *lda, int dtype,
                           tsqr_batch_plan_t *plan);
int tsqr_batch_plan_destroy(tsqr_batch_plan_t plan);

/* Workspace bytes for tsqr_batch_exec (tree counters and triangles of all
 * instances), or -1 for a NULL plan. */
int64_t tsqr_batch_workspace_bytes(tsqr_batch_plan_t plan);

/* Tiles (workgroups), leaves over all instances and rows per leaf. */
int tsqr_batch_plan_info(tsqr_batch_plan_t plan, int64_t *tiles, int64_t *leaves, int64_t *leaf_rows);

/* The schedule the plan launches, copied to host arrays (for checks; the
 * device copies are what exec uses).  inst: 7 values per instance b at
 * inst[7b]: element offset of A, m, lda, leaf rows, leaf count, index of its
 * first tree counter, element offset of its first triangle slot.  tiles: 2
 * values per workgroup t in launch order at tiles[2t]: (instance, leaf),
 * longest leaves first, ties in instance order.  Either pointer may be NULL
 * (sizes from tsqr_batch_plan_info).  Returns 0, or -1 for a NULL plan. */
int tsqr_batch_plan_schedule(tsqr_batch_plan_t plan, int64_t *inst, int64_t *tiles);

/* R of every instance: instance b's n-by-n R (diag >= 0, column-major,
 * leading dimension ldr >= n) is written at R + b*ldr*n elements.  A and R
 * are device pointers of the plan's element type; ws as for tsqr_geqr_r_*.
 * Argument codes: -1 plan, -2 A, -3 R, -4 ldr, -5 ws, -6 ws_bytes. */
int tsqr_batch_exec(tsqr_batch_plan_t plan, const void *A, void *R, int64_t ldr, void *ws, int64_t ws_bytes,
                    void *stream);

/* tsqr_batch_exec that also measures its schedule: workgroup g (tile g of the
 * plan's longest-first order, tsqr_batch_plan_info's tile count) writes the
 * device's constant-rate clock when it starts and when it is done (its leaf
 * and the merges it performed) to stamps[2g] and stamps[2g + 1] (device
 * memory, 2 x tiles values, owned by the caller; ticks at
 * tsqr_device_clock_khz kHz, arbitrary origin).  R is bit-identical to
 * tsqr_batch_exec's.  Argument codes as tsqr_batch_exec's, plus -7 stamps. */
int tsqr_batch_exec_stamped(tsqr_batch_plan_t plan, const void *A, void *R, int64_t ldr, void *ws, int64_t ws_bytes,
                            uint64_t *stamps, void *stream);

/* The rate of the clock of tsqr_batch_exec_stamped, in kHz (> 0); -1 for a
 * NULL handle, -1000 - status otherwise (TSQR_ERR_NO_DEVICE on a planning
 * handle, TSQR_ERR_HIP if the runtime cannot tell). */
int64_t tsqr_device_clock_khz(tsqr_handle_t handle);

/* ---- the Q factor --------------------------------------------------------------
 *
 * A = Q R with Q m x n with orthonormal columns (column-major, ldq >= m) and R
 * as tsqr_geqr_r_f64 / _f32 returns it (same leaf size, bit-identical R),
 * m >= n.  The factorization keeps every reflector it applies (leaf
 * reflectors, and the V and tau of every merge of the tree, Table 3's
 * outputs), and Q is formed from them: one pass down the tree, one launch per
 * level, then one pass over the leaves (the implicit Q of section 3, made
 * explicit).  Rows per lane are fixed at 8 for this mode (128-row chunks).
 * A, Q, R and ws are device pointers owned by the caller; the call is
 * asynchronous on `stream` and allocates nothing.  The workspace (256-byte
 * aligned) holds the reflector block, m rounded up to whole chunks by n, so it
 * is about m*n elements larger than tsqr_geqr_r's.
 *
 * tsqr_qr_workspace_bytes: bytes for (m, n, dtype); negative for bad
 * arguments: -1 handle, -2 m, -3 n (n > m is illegal), -4 dtype, and
 * -1000 - status for a planning failure.
 * tsqr_geqr_qr_*: argument codes -1 handle, -2 m, -3 n (n > m is illegal),
 * -4 A, -5 lda, -6 Q, -7 ldq, -8 R, -9 ldr, -10 ws, -11 ws_bytes;
 * TSQR_ERR_UNSUPPORTED for n > TSQR_MAX_N. */
int64_t tsqr_qr_workspace_bytes(tsqr_handle_t handle, int64_t m, int64_t n, int dtype);
int tsqr_geqr_qr_f64(tsqr_handle_t handle, int64_t m, int64_t n, const double *A, int64_t lda, double *Q,
                     int64_t ldq, double *R, int64_t ldr, void *ws, int64_t ws_bytes, void *stream);
int tsqr_geqr_qr_f32(tsqr_handle_t handle, int64_t m, int64_t n, const float *A, int64_t lda, float *Q,
                     int64_t ldq, float *R, int64_t ldr, void *ws, int64_t ws_bytes, void *stream);

/* Applying Q^T without forming Q (section 3: Q stays implicit in the leaves'
 * and the tree's reflectors).  tsqr_geqrf_* is the factorization of
 * tsqr_geqr_qr_* alone: it returns R (bit-identical to tsqr_geqr_r's with the
 * same leaf size) and leaves every reflector in ws; argument codes -1 handle,
 * -2 m, -3 n (n > m is illegal), -4 A, -5 lda, -6 R, -7 ldr, -8 ws,
 * -9 ws_bytes.  tsqr_apply_qt_* then computes C = Q^T B (n x k, column-major,
 * ldc >= n) for any B (m x k, column-major, ldb >= m), k >= 0, by replaying
 * those reflectors on B in the factorization's order: each leaf maps its rows
 * of B chunk by chunk into an n x k block, the tree's merges combine the
 * blocks level by level from the leaves up, and the root's sign flips finish
 * it.  It must follow a tsqr_geqrf_* call of the same precision with the same
 * handle, m, n and ws, whose contents it reads and does not change, so any
 * number of right-hand sides can follow one factorization (tsqr_geqr_qr_*
 * overwrites part of that state while forming Q).  ws is sized by
 * tsqr_qr_workspace_bytes, which includes the per-leaf blocks for k.  k is
 * taken in panels of 48 columns in FP64, 64 in FP32 (a separate kernel for
 * k <= 4).  Asynchronous on `stream`, no allocation.  Argument codes -1
 * handle, -2 m, -3 n, -4 k, -5 B, -6 ldb, -7 C, -8 ldc, -9 ws, -10 ws_bytes;
 * TSQR_ERR_UNSUPPORTED for n > TSQR_MAX_N. */
int tsqr_geqrf_f64(tsqr_handle_t handle, int64_t m, int64_t n, const double *A, int64_t lda, double *R, int64_t ldr,
                   void *ws, int64_t ws_bytes, void *stream);
int tsqr_geqrf_f32(tsqr_handle_t handle, int64_t m, int64_t n, const float *A, int64_t lda, float *R, int64_t ldr,
                   void *ws, int64_t ws_bytes, void *stream);
int tsqr_apply_qt_f64(tsqr_handle_t handle, int64_t m, int64_t n, int64_t k, const double *B, int64_t ldb, double *C,
                      int64_t ldc, void *ws, int64_t ws_bytes, void *stream);
int tsqr_apply_qt_f32(tsqr_handle_t handle, int64_t m, int64_t n, int64_t k, const float *B, int64_t ldb, float *C,
                      int64_t ldc, void *ws, int64_t ws_bytes, void *stream);

/* ---- mixed precision: FP32 TSQR, then one FP64 correction -------------------
 *
 * For `batch` matrices of equal shape m x n stored in FP32 (instance b at
 * A + b*stride_a, column-major, leading dimension lda), R with FP64 accuracy:
 * the FP32 batched TSQR (section 2 of the paper in FP32) gives R~; one FP64
 * pass over A then forms Y = A R~^-1 and G = Y^T Y and returns
 * R = chol(G) R~, the second pass of CholeskyQR2 (Fukaya, Nakatsukasa,
 * Yanagisawa, Yamamoto 2014) with the Householder factorization as its first
 * pass.  It is accurate while kappa(A) * 2^-24 << 1 and G stays numerically
 * positive definite.  An instance whose Cholesky factorization meets a pivot
 * that is not positive and finite (an exactly or numerically rank-deficient
 * R~; no instance of uniform or conditioned test matrices up to kappa = 1e8 has
 * needed it) is refactored by the plain FP64 TSQR path, which reads its FP32
 * storage directly; that decision is taken on the device.
 *
 * Create: argument codes -1 handle, -2 batch, -3 m, -4 n, -5 lda, -6 stride_a,
 * -7 plan; the plan holds two batched plans (the FP32 factorization and the
 * FP64 fallback, both with the geometry fixed at creation: later option or
 * tuning changes on the handle do not affect it), four small device tables.
 * Exec: R is FP64, instance b's n x n R (diag >= 0) at R + b*ldr*n;
 * `fallback` is NULL or a DEVICE array of `batch` ints, written on `stream`
 * (1 = the instance took the FP64 path; every instance when m = 0).  The call
 * is asynchronous on `stream`: kernel launches only, no host synchronization,
 * no allocation, no memset, so it can be captured in a HIP graph.  Argument
 * codes -1 plan, -2 A, -3 R, -4 ldr, -6 ws, -7 ws_bytes. */
int tsqr_mixed_plan_create(tsqr_handle_t handle, int64_t batch, int64_t m, int64_t n, int64_t lda,
                           int64_t stride_a, tsqr_mixed_plan_t *plan);
int tsqr_mixed_plan_destroy(tsqr_mixed_plan_t plan);
int64_t tsqr_mixed_workspace_bytes(tsqr_mixed_plan_t plan);
int tsqr_mixed_exec(tsqr_mixed_plan_t plan, const float *A, double *R, int64_t ldr, int *fallback, void *ws,
                    int64_t ws_bytes, void *stream);

/* The same plan with R~ computed from a row sample instead of all of A (the
 * sampled preconditioner: the paper's method is unchanged in the fallback,
 * only the preconditioner of the FP64 pass is cheaper).  The sample has
 * sample_rows rows rounded up to a multiple of 64: the m rows are cut into
 * sample_rows/64 strata of equal length (to within one row), and from each a
 * block of 64 contiguous rows at a uniform offset is taken, the offsets drawn
 * from SplitMix64 (Steele, Lea and Flood 2014) of (seed, instance, stratum),
 * so a plan always takes the same sample.  The FP32 TSQR then factors the
 * sample, and the FP64 pass over all of A corrects as above: the result is
 * the R of A, whatever the sample, whenever the Cholesky factorization
 * succeeds (the sample only has to make A R~^-1 well conditioned), and the
 * plain FP64 path otherwise.  sample_rows = 0, or a rounded count of at least
 * m, makes it the plain mixed plan.  Argument codes as for the plain create,
 * plus -7 sample_rows < 0, -9 plan.  Exec, destroy and workspace as above. */
int tsqr_mixed_plan_create_sampled(tsqr_handle_t handle, int64_t batch, int64_t m, int64_t n, int64_t lda,
                                   int64_t stride_a, int64_t sample_rows, uint64_t seed, tsqr_mixed_plan_t *plan);

/* The correction with the caller's R~ (device, FP32, instance b's n x n upper
 * triangle at Rt + b*n*n, column-major, ld n) instead of the plan's own FP32
 * factorization (e.g. a learned correction of the sampled R~, below): the
 * FP64 pass, the guards and the fallback are those of tsqr_mixed_exec, so the
 * result is the R of A whatever R~ is.  Argument codes as tsqr_mixed_exec's
 * with -3 for Rt and the later ones one lower (-4 R, -5 ldr, -7 ws, -8
 * ws_bytes). */
int tsqr_mixed_exec_rtilde(tsqr_mixed_plan_t plan, const float *A, const float *Rt, double *R, int64_t ldr,
                           int *fallback, void *ws, int64_t ws_bytes, void *stream);

/* Only the first stage of tsqr_mixed_exec: R~ by the FP32 TSQR of A (or of its
 * row sample, for a sampled plan), left in the workspace at
 * tsqr_mixed_rtilde_offset (e.g. as the input of a learned correction, whose
 * result then goes to tsqr_mixed_exec_rtilde).  Nothing is written for m = 0.
 * Argument codes: -1 plan, -2 A, -3 ws (NULL or not 256-byte aligned), -4
 * ws_bytes; TSQR_ERR_NO_DEVICE on a planning handle. */
int tsqr_mixed_rtilde_exec(tsqr_mixed_plan_t plan, const float *A, void *ws, int64_t ws_bytes, void *stream);

/* Byte offset in the workspace of R~ after tsqr_mixed_exec: FP32, instance b's
 * n x n upper triangle at offset + 4*b*n*n, column-major, ld n (for
 * diagnostics such as the conditioning of A R~^-1); -1 for a NULL plan. */
int64_t tsqr_mixed_rtilde_offset(tsqr_mixed_plan_t plan);

/* ---- the learned correction of the sampled preconditioner -------------------
 *
 * The slot where a model can enter without changing the result is R~ (above):
 * these calls are the building blocks of a small MLP that maps features of a
 * sampled R~ to a correction of it, trained on the GPU.  All arrays are device
 * FP32, column-major with the given leading dimension, owned by the caller;
 * every call is asynchronous on `stream` and allocates nothing.  The paper has
 * no learned part: these calls serve the preconditioner above only.  Sizes are
 * below 2^31.  A call whose output is empty (M or N, rows or cols, count or
 * batch 0) returns 0 without a launch; tsqr_mlp_colsum with no rows writes
 * zero sums, tsqr_gemm_bf16 with K = 0 writes beta C, and tsqr_mlp_mse needs
 * rows, cols >= 1.  n is 1..TSQR_MAX_N for the feature, target and correction
 * maps.  Argument
 * codes: -k for the k-th argument; TSQR_ERR_NO_DEVICE on a planning handle.
 *
 * tsqr_gemm_bf16: C (M x N, ldc) = alpha op(A) op(B) + beta C with op(X) = X or
 *   X^T (ta, tb nonzero: stored transposed; op(A) is M x K, op(B) K x N).  A
 *   and B are rounded to BF16 as they are loaded (round to nearest even), the
 *   products accumulate in FP32 on the BF16 matrix cores (the 16x16x16 BF16
 *   instruction); beta = 0 does not read C.
 * tsqr_mlp_bias_act: Z (rows x cols, ld) := act(Z + bias), bias per column, act
 *   ReLU if relu is nonzero, else the identity.
 * tsqr_mlp_relu_grad: dA := dA where out > 0, else 0 (out: the ReLU output).
 * tsqr_mlp_colsum: s(j) = sum over the rows of Z(:, j), in row order.
 * tsqr_mlp_mse: D = 2 (Y - T)/(rows cols) and *loss = sum (Y - T)^2/(rows cols)
 *   (loss: one device float), in a fixed order.
 * tsqr_mlp_adam: one Adam step (Kingma and Ba 2015) on count parameters, step
 *   >= 1 for the bias corrections.
 * tsqr_surrogate_features: for a batch of R~ (instance b at Rt + b*n*n, ld n),
 *   X (batch x (2n - 1), ld batch): log|R~(i,i)| minus its mean over i, then
 *   R~(i-1, i)/|R~(i-1, i-1)| for i = 1..n-1.  A zero diagonal entry makes
 *   the instance's features non-finite; the correction then clamps what the
 *   network gives (below), and the guard of the FP64 pass decides.
 * tsqr_surrogate_targets: Y (batch x n, ld batch) = log(|R(i,i)|/|R~(i,i)|)
 *   minus its mean over i, R the FP64 R of all of A (instance b at R + b*ldr*n).
 * tsqr_surrogate_apply: Rout = R~ with row i scaled by exp(Y(b, i)), Y(b, i)
 *   clamped to [-1, 1] (a NaN to -1): no row changes by more than a factor e. */
int tsqr_gemm_bf16(tsqr_handle_t handle, int ta, int tb, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                   int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc, void *stream);
int tsqr_mlp_bias_act(tsqr_handle_t handle, float *Z, int64_t rows, int64_t cols, int64_t ld, const float *bias,
                      int relu, void *stream);
int tsqr_mlp_relu_grad(tsqr_handle_t handle, float *dA, const float *out, int64_t rows, int64_t cols, int64_t ld,
                       void *stream);
int tsqr_mlp_colsum(tsqr_handle_t handle, const float *Z, int64_t rows, int64_t cols, int64_t ld, float *s,
                    void *stream);
int tsqr_mlp_mse(tsqr_handle_t handle, const float *Y, const float *T, float *D, int64_t rows, int64_t cols,
                 int64_t ld, float *loss, void *stream);
int tsqr_mlp_adam(tsqr_handle_t handle, float *p, const float *g, float *m, float *v, int64_t count, float lr,
                  float b1, float b2, float eps, int64_t step, void *stream);
int tsqr_surrogate_features(tsqr_handle_t handle, const float *Rt, int64_t batch, int64_t n, float *X, void *stream);
int tsqr_surrogate_targets(tsqr_handle_t handle, const double *R, int64_t ldr, const float *Rt, int64_t batch,
                           int64_t n, float *Y, void *stream);
int tsqr_surrogate_apply(tsqr_handle_t handle, const float *Rt, const float *Y, int64_t batch, int64_t n, float *Rout,
                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_H */
