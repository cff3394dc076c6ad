/*
 * tsqr_oracle.c -- CPU oracle for the R factor of a tall-skinny QR.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded IEEE double code
 * that the tests, the package smoke check and the benchmark's CPU-baseline leg
 * use to check the GPU library.  It shares no code, header, table or helper
 * with the GPU path and must never be linked into it or called by it.
 *
 * Source: J. Langou, "Computing the R of the QR factorization of tall and
 * skinny matrices using MPI_Reduce" (arXiv:1002.4250).
 *
 *   oracle_r_factor        -- the plain definition: the upper-triangular R of
 *                             A = QR (Q orthonormal columns) with a
 *                             non-negative diagonal (section 2: R is unique up
 *                             to the sign of each row; fixing the diagonal
 *                             sign makes it unique).  Computed by textbook
 *                             column-by-column Householder QR of all of A.
 *   oracle_reflector       -- elementary Householder reflector generation, as
 *                             used for every column step of the operator
 *                             (Table 3 builds each reflector this way).
 *   oracle_qr_uppers       -- the paper's reduction operator R := qr(R1, R2)
 *                             on two n-by-n upper triangles, with the output
 *                             contract of section 3 / Table 3: R overwrites R1,
 *                             the Householder vectors V (upper triangular,
 *                             reflectors represented as [I; V]) overwrite R2,
 *                             and tau holds the n reflector scalars.
 *   oracle_tsqr_r          -- the method itself (section 2, Table 1): local
 *                             Householder QR of each row block (step 1), then
 *                             a reduction of the block triangles with
 *                             qr_uppers (step 2) over a chosen tree, then the
 *                             sign normalisation.
 *   oracle_normalize_signs -- flip every row whose diagonal entry has its
 *                             sign bit set (section 2, positive-diagonal
 *                             convention).
 *   oracle_q_factor        -- the plain definition of the Q that goes with
 *                             that R: for A of full column rank, Q = A R^-1
 *                             is the unique m-by-n matrix with orthonormal
 *                             columns and A = QR, diag(R) > 0 (the Q that
 *                             section 3 notes a reduction leaves implicit).
 *   oracle_gram            -- the Gram matrix A^T A, each entry summed in
 *                             double-double arithmetic from exact products
 *                             (the identity R^T R = A^T A that every R of
 *                             section 2 satisfies, whatever the tree).
 *   oracle_gram_residual   -- ||R^T R - A^T A||_F / ||A||_F^2 with both Gram
 *                             matrices and their difference carried in
 *                             double-double: the backward error of a
 *                             computed R, accurate far below FP64 rounding.
 *
 * Storage is column-major throughout: element (i, j) of a matrix with leading
 * dimension ld sits at index i + j*ld.  Return value 0 means success; a
 * negative value -k means argument k was invalid.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((int64_t)(i) + (int64_t)(j) * (int64_t)(ld))

/* Compensated (Neumaier) running sum: the pair (s, c) carries the sum and
 * the rounding error lost so far, so the result's error does not grow with the
 * number of terms.  Keeps the oracle's own error far below the GPU's even for
 * m = 2^22 rows. */
typedef struct { double s, c; } csum_t;

static void csum_add(csum_t *a, double t)
{
    double u = a->s + t;
    if (fabs(a->s) >= fabs(t)) a->c += (a->s - u) + t;
    else a->c += (t - u) + a->s;
    a->s = u;
}

static double csum_value(const csum_t *a) { return a->s + a->c; }

/* Euclidean norm of x[0], x[inc], ..., x[(len-1)*inc] without intermediate
 * overflow or underflow: every entry is first scaled by the power of two 2^-e
 * that brings the largest magnitude into [0.5, 1) (an exact scaling), the
 * squares are summed with compensation, and the root is scaled back. */
static double scaled_norm2(int64_t len, const double *x, int64_t inc)
{
    double amax = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double a = fabs(x[i * inc]);
        if (isnan(a)) return a;
        if (a > amax) amax = a;
    }
    if (amax == 0.0 || isinf(amax)) return amax;
    int e;
    frexp(amax, &e);
    csum_t acc = {0.0, 0.0};
    for (int64_t i = 0; i < len; ++i) {
        double t = ldexp(x[i * inc], -e);
        csum_add(&acc, t * t);
    }
    return ldexp(sqrt(csum_value(&acc)), e);
}

/* Elementary reflector (section 3 and Table 3 generate each column's reflector
 * this way).  Given alpha and the vector x (len-1 entries, stride incx), find
 * beta, tau and v with
 *     H^T [alpha; x] = [beta; 0],   H = I - tau [1; v] [1; v]^T,
 * beta = -sign(alpha) * ||[alpha; x]||.  On return *alpha = beta and x holds v.
 * If x is zero the reflector is the identity: tau = 0 and alpha is kept.  The
 * sign of alpha is read from its sign bit, so alpha = -0.0 counts as negative. */
int oracle_reflector(int64_t len, double *alpha, double *x, int64_t incx, double *tau)
{
    if (len < 1) return -1;
    if (!alpha) return -2;
    if (len > 1 && !x) return -3;
    if (!tau) return -5;
    *tau = 0.0;
    if (len == 1) return 0;
    double xnorm = scaled_norm2(len - 1, x, incx);
    if (xnorm == 0.0) return 0;
    double a = *alpha;
    double nrm = hypot(a, xnorm);
    /* Tiny norms (below the smallest normal number over machine epsilon, the
     * reflector generator's usual safe minimum): 1/(alpha - beta) would
     * overflow, so alpha and x are first scaled up by an exact power of two.
     * tau and v do not change under that scaling; beta is scaled back.  Such
     * norms arise for the roundoff left in rank-deficient triangles, e.g. a
     * block with fewer rows than columns. */
    int shift = 0;
    if (nrm < DBL_MIN / DBL_EPSILON) {
        int e;
        frexp(nrm, &e);
        shift = -e;
        a = ldexp(a, shift);
        for (int64_t i = 0; i < len - 1; ++i) x[i * incx] = ldexp(x[i * incx], shift);
        nrm = hypot(a, scaled_norm2(len - 1, x, incx));
    }
    double beta = signbit(a) ? nrm : -nrm;
    *tau = (beta - a) / beta;
    double scal = 1.0 / (a - beta);
    for (int64_t i = 0; i < len - 1; ++i) x[i * incx] *= scal;
    *alpha = ldexp(beta, -shift);
    return 0;
}

/* Householder QR of the m-by-n matrix A in place, one column at a time:
 * on return the upper triangle of A(0:min(m,n)-1, :) holds R (unnormalised
 * signs) and tau[0..min(m,n)-1] the reflector scalars; the Householder vectors
 * are left below the diagonal.  This is the local factorisation of step 1
 * (section 3; any Householder variant yields the same R up to rounding). */
static void householder_inplace(int64_t m, int64_t n, double *A, int64_t lda, double *tau)
{
    int64_t kmax = m < n ? m : n;
    for (int64_t j = 0; j < kmax; ++j) {
        double *ajj = &A[IDX(j, j, lda)];
        double *x = (j + 1 < m) ? &A[IDX(j + 1, j, lda)] : NULL;
        oracle_reflector(m - j, ajj, x, 1, &tau[j]);
        if (tau[j] == 0.0) continue;
        for (int64_t k = j + 1; k < n; ++k) {
            double *ak = &A[IDX(0, k, lda)];
            /* w = tau [1; v]^T A(j:m-1, k), the dot product summed with compensation */
            csum_t acc = {ak[j], 0.0};
            for (int64_t i = j + 1; i < m; ++i) csum_add(&acc, A[IDX(i, j, lda)] * ak[i]);
            double w = tau[j] * csum_value(&acc);
            ak[j] -= w;
            for (int64_t i = j + 1; i < m; ++i) ak[i] -= w * A[IDX(i, j, lda)];
        }
    }
}

/* Row sign normalisation (section 2): multiply row i of the upper-triangular
 * n-by-n R by -1 when the sign bit of R(i,i) is set, so the diagonal becomes
 * >= +0.  Only the upper part (columns i..n-1) is touched, so the zeros below
 * the diagonal stay +0.0. */
void oracle_normalize_signs(int64_t n, double *R, int64_t ldr)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!signbit(R[IDX(i, i, ldr)])) continue;
        for (int64_t j = i; j < n; ++j) R[IDX(i, j, ldr)] = -R[IDX(i, j, ldr)];
    }
}

/* Copy the upper triangle of the leading min(m,n)-by-n block of A into the
 * n-by-n R (zero below the diagonal and in rows m..n-1 when m < n). */
static void extract_upper(int64_t m, int64_t n, const double *A, int64_t lda, double *R, int64_t ldr)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            R[IDX(i, j, ldr)] = (i <= j && i < m) ? A[IDX(i, j, lda)] : 0.0;
}

/* The plain definition: R of A = QR with diag(R) >= 0, computed by
 * Householder QR of the whole of A (A itself is not modified).
 * R is n-by-n column-major with leading dimension ldr >= max(1,n). */
int oracle_r_factor(int64_t m, int64_t n, const double *A, int64_t lda, double *R, int64_t ldr)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && n > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (n > 0 && !R) return -5;
    if (ldr < (n > 1 ? n : 1)) return -6;
    if (n == 0) return 0;
    if (m == 0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = 0.0;
        return 0;
    }
    double *W = (double *)malloc(sizeof(double) * (size_t)m * (size_t)n);
    double *tau = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!W || !tau) { free(W); free(tau); return 1; }
    for (int64_t j = 0; j < n; ++j) memcpy(&W[IDX(0, j, m)], &A[IDX(0, j, lda)], sizeof(double) * (size_t)m);
    householder_inplace(m, n, W, m, tau);
    extract_upper(m, n, W, m, R, ldr);
    oracle_normalize_signs(n, R, ldr);
    free(W);
    free(tau);
    return 0;
}

/* The Q of A = QR for A of full column rank with diag(R) > 0: Q = A R^-1 with
 * R from oracle_r_factor.  Each row q of Q solves q R = a (a the row of A) by
 * forward substitution over the columns, q_j = (a_j - sum_{i<j} q_i R(i,j)) /
 * R(j,j), with compensated sums.  Q is m-by-n column-major, ldq >= max(1,m);
 * m >= n.  Returns 2 if a diagonal entry of R is zero (rank deficient: Q is
 * not unique) and 1 if memory runs out. */
int oracle_q_factor(int64_t m, int64_t n, const double *A, int64_t lda, double *Q, int64_t ldq)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (n > 0 && !Q) return -5;
    if (ldq < (m > 1 ? m : 1)) return -6;
    if (n == 0) return 0;
    double *R = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    if (!R) return 1;
    int rc = oracle_r_factor(m, n, A, lda, R, n);
    if (rc) { free(R); return rc; }
    for (int64_t j = 0; j < n; ++j) {
        if (!(R[IDX(j, j, n)] > 0.0)) { free(R); return 2; }
    }
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t j = 0; j < n; ++j) {
            csum_t acc = {A[IDX(r, j, lda)], 0.0};
            for (int64_t i = 0; i < j; ++i) csum_add(&acc, -Q[IDX(r, i, ldq)] * R[IDX(i, j, n)]);
            Q[IDX(r, j, ldq)] = csum_value(&acc) / R[IDX(j, j, n)];
        }
    }
    free(R);
    return 0;
}

/* The reduction operator of section 2, R := qr([R1; R2]) for two n-by-n upper
 * triangles, exploiting that both inputs are triangular (Table 3; cost 2/3 n^3).
 * For column j = 0..n-1, with 0-based indices:
 *   1. the reflector for the (j+2)-vector [R1(j,j); R2(0:j, j)] is generated:
 *      R1(j,j) becomes beta, R2(0:j, j) becomes its vector v, tau[j] its scalar;
 *   2. if j < n-1 and tau[j] != 0, the reflector is applied to the trailing
 *      columns: w := R2(0:j, j+1:n-1)^T v + R1(j, j+1:n-1)^T,
 *      R1(j, j+1:n-1) -= tau[j] w^T,  R2(0:j, j+1:n-1) -= tau[j] v w^T.
 * On return R1 holds R (diagonal signs as the reflectors leave them), R2 holds
 * the upper-triangular V, and tau the n scalars.  Both matrices are n-by-n
 * column-major with leading dimension n. */
int oracle_qr_uppers(int64_t n, double *R1, double *R2, double *tau)
{
    if (n < 0) return -1;
    if (n > 0 && (!R1)) return -2;
    if (n > 0 && (!R2)) return -3;
    if (n > 0 && (!tau)) return -4;
    double *w = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!w) return 1;
    for (int64_t j = 0; j < n; ++j) {
        double *v = &R2[IDX(0, j, n)];
        /* reflector of length j+2: alpha = R1(j,j), x = R2(0:j, j) */
        oracle_reflector(j + 2, &R1[IDX(j, j, n)], v, 1, &tau[j]);
        if (j == n - 1 || tau[j] == 0.0) continue;
        for (int64_t k = j + 1; k < n; ++k) {
            double s = 0.0;
            for (int64_t i = 0; i <= j; ++i) s += R2[IDX(i, k, n)] * v[i];
            w[k] = s + R1[IDX(j, k, n)];
        }
        for (int64_t k = j + 1; k < n; ++k) {
            double t = tau[j] * w[k];
            R1[IDX(j, k, n)] -= t;
            for (int64_t i = 0; i <= j; ++i) R2[IDX(i, k, n)] -= v[i] * t;
        }
    }
    free(w);
    return 0;
}

/* Local factorisation of one row block (step 1): rows [r0, r1) of A, all n
 * columns, Householder QR without sign normalisation; the n-by-n triangle goes
 * to T (leading dimension n; zero rows beyond the block's row count). */
static int leaf_triangle(int64_t r0, int64_t r1, int64_t n, const double *A, int64_t lda, double *T)
{
    int64_t b = r1 - r0;
    int64_t rows = b > 0 ? b : 1;
    double *W = (double *)calloc((size_t)rows * (size_t)n, sizeof(double));
    double *tau = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!W || !tau) { free(W); free(tau); return 1; }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < b; ++i) W[IDX(i, j, rows)] = A[IDX(r0 + i, j, lda)];
    householder_inplace(b, n, W, rows, tau);
    extract_upper(b, n, W, rows, T, n);
    free(W);
    free(tau);
    return 0;
}

/* R := qr(Ra, Rb) with Ra on top, result left in Ra (Rb is overwritten by V). */
static int merge_into(int64_t n, double *Ra, double *Rb, double *tau)
{
    return oracle_qr_uppers(n, Ra, Rb, tau);
}

/* The method (section 2, Table 1): split the rows of A into blocks of
 * leaf_rows rows (the last block may be shorter), factor each block
 * (step 1), and reduce the block triangles with qr_uppers (step 2):
 *   tree = 0: binary tree, level l pairs block i with block i + 2^l, the lower
 *             index on top (the hand-made binary tree of section 4);
 *   tree = 1: flat tree, R := qr(R, R_i) for i = 1, 2, ... in order;
 *   tree = 2: flat tree with the operands swapped, R := qr(R_i, R)
 *             (the operator is essentially commutative, section 2);
 *   tree = 3: flat tree over the block order given by perm[0..P-1]
 *             (a permutation of 0..P-1; any tree is allowed, section 2).
 * Finally the diagonal signs are normalised.  R is n-by-n, leading dimension
 * ldr. */
int oracle_tsqr_r(int64_t m, int64_t n, const double *A, int64_t lda, int64_t leaf_rows,
                  int tree, const int64_t *perm, double *R, int64_t ldr)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && n > 0 && !A) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (leaf_rows < 1) return -5;
    if (tree < 0 || tree > 3) return -6;
    if (tree == 3 && !perm) return -7;
    if (n > 0 && !R) return -8;
    if (ldr < (n > 1 ? n : 1)) return -9;
    if (n == 0) return 0;
    int64_t P = m > 0 ? (m + leaf_rows - 1) / leaf_rows : 1;
    size_t tri = (size_t)n * (size_t)n;
    double *T = (double *)calloc((size_t)P * tri, sizeof(double));
    double *tau = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!T || !tau) { free(T); free(tau); return 1; }
    int rc = 0;
    for (int64_t p = 0; p < P && rc == 0; ++p) {
        int64_t r0 = p * leaf_rows, r1 = r0 + leaf_rows;
        if (r1 > m) r1 = m;
        rc = leaf_triangle(r0, r1, n, A, lda, &T[(size_t)p * tri]);
    }
    int64_t root = 0;
    if (rc == 0 && tree == 0) {
        for (int64_t step = 1; step < P && rc == 0; step *= 2)
            for (int64_t i = 0; i + step < P && rc == 0; i += 2 * step)
                rc = merge_into(n, &T[(size_t)i * tri], &T[(size_t)(i + step) * tri], tau);
    } else if (rc == 0 && tree == 1) {
        for (int64_t i = 1; i < P && rc == 0; ++i) rc = merge_into(n, &T[0], &T[(size_t)i * tri], tau);
    } else if (rc == 0 && tree == 2) {
        /* acc lives in block 0's slot; qr(R_i, acc) leaves the result in R_i's slot */
        int64_t acc = 0;
        for (int64_t i = 1; i < P && rc == 0; ++i) {
            rc = merge_into(n, &T[(size_t)i * tri], &T[(size_t)acc * tri], tau);
            acc = i;
        }
        root = acc;
    } else if (rc == 0 && tree == 3) {
        for (int64_t i = 0; i < P; ++i)
            if (perm[i] < 0 || perm[i] >= P) { rc = -7; break; }
        if (rc == 0) {
            root = perm[0];
            for (int64_t i = 1; i < P && rc == 0; ++i)
                rc = merge_into(n, &T[(size_t)root * tri], &T[(size_t)perm[i] * tri], tau);
        }
    }
    if (rc == 0) {
        const double *Rt = &T[(size_t)root * tri];
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = i <= j ? Rt[IDX(i, j, n)] : 0.0;
        oracle_normalize_signs(n, R, ldr);
    }
    free(T);
    free(tau);
    return rc;
}

/* Operation count of oracle_tsqr_r in the paper's flop model (section 2 and
 * Table 3): a length-L Householder step applied to K trailing columns costs
 * 4*L*K flops (dot products plus the rank-1 update), the same model that gives
 * 2mn^2 - 2/3 n^3 for a full QR and 2/3 n^3 for one qr_uppers.  Counts the leaf
 * factorisations plus P-1 merges; independent of the tree shape. */
double oracle_tsqr_flops(int64_t m, int64_t n, int64_t leaf_rows)
{
    if (m <= 0 || n <= 0 || leaf_rows < 1) return 0.0;
    int64_t P = (m + leaf_rows - 1) / leaf_rows;
    double total = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        int64_t b = (p == P - 1) ? m - p * leaf_rows : leaf_rows;
        int64_t kmax = b < n ? b : n;
        for (int64_t j = 0; j < kmax; ++j) total += 4.0 * (double)(b - j) * (double)(n - 1 - j);
    }
    for (int64_t p = 1; p < P; ++p)
        for (int64_t j = 0; j < n; ++j) total += 4.0 * (double)(j + 1) * (double)(n - 1 - j);
    return total;
}

/* ---- Gram matrices in double-double ---------------------------------------
 *
 * A double-double value is an unevaluated sum hi + lo with |lo| <= ulp(hi)/2.
 * two_sum and two_prod are the error-free transformations of Knuth and
 * Dekker (the product's rounding error is exact through fma), so a dot product
 * accumulated this way carries an error of order 2^-104 relative to the sum
 * of |terms|, independent of the number of terms. */
typedef struct { double hi, lo; } dd_t;

static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

static void dd_add_prod(dd_t *acc, double a, double b)
{
    double p = a * b;
    double pe = fma(a, b, -p);       /* a*b = p + pe exactly */
    double s, e;
    two_sum(acc->hi, p, &s, &e);
    e += acc->lo + pe;
    two_sum(s, e, &acc->hi, &acc->lo);
}

static dd_t dd_sub(dd_t a, dd_t b)
{
    double s, e;
    two_sum(a.hi, -b.hi, &s, &e);
    e += a.lo - b.lo;
    dd_t r;
    two_sum(s, e, &r.hi, &r.lo);
    return r;
}

/* The upper triangle (j <= k) of X^T X for an m-by-n X in double-double,
 * packed by rows of the triangle into acc[0 .. n(n+1)/2).  Rows of X are taken
 * one at a time (through a small row buffer), so every accumulator of the row
 * is independent of the others and the loop pipelines. */
static int gram_dd(int64_t m, int64_t n, const double *X, int64_t ldx, dd_t *acc)
{
    double *row = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!row) return -1;
    int64_t nt = n * (n + 1) / 2;
    for (int64_t t = 0; t < nt; ++t) acc[t].hi = acc[t].lo = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) row[j] = X[IDX(i, j, ldx)];
        dd_t *a = acc;
        for (int64_t j = 0; j < n; ++j) {
            double xj = row[j];
            for (int64_t k = j; k < n; ++k) dd_add_prod(a++, xj, row[k]);
        }
    }
    free(row);
    return 0;
}

/* G = A^T A (n-by-n, leading dimension ldg), each entry rounded once from its
 * double-double sum. */
int oracle_gram(int64_t m, int64_t n, const double *A, int64_t lda, double *G, int64_t ldg)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (ldg < (n > 1 ? n : 1)) return -6;
    dd_t *acc = (dd_t *)malloc((size_t)(n * (n + 1) / 2 + 1) * sizeof(dd_t));
    if (!acc) return -7;
    if (gram_dd(m, n, A, lda, acc) != 0) {
        free(acc);
        return -7;
    }
    const dd_t *a = acc;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = j; k < n; ++k, ++a) G[IDX(j, k, ldg)] = G[IDX(k, j, ldg)] = a->hi + a->lo;
    free(acc);
    return 0;
}

/* ||R^T R - A^T A||_F / ||A||_F^2 for an m-by-n A and an n-by-n R (only its
 * upper triangle is read).  Both Gram matrices and each difference are formed
 * in double-double; the norms are summed from the rounded differences.
 * Returns -1 if A is zero (result undefined), -2 for bad sizes or no memory,
 * else the ratio. */
double oracle_gram_residual(int64_t m, int64_t n, const double *A, int64_t lda, const double *R, int64_t ldr)
{
    if (m < 0 || n < 0 || lda < (m > 1 ? m : 1) || ldr < (n > 1 ? n : 1)) return -2.0;
    int64_t nt = n * (n + 1) / 2;
    dd_t *ga = (dd_t *)malloc((size_t)(nt + 1) * sizeof(dd_t));
    dd_t *gr = (dd_t *)malloc((size_t)(nt + 1) * sizeof(dd_t));
    double *Ru = (double *)calloc((size_t)(n * n + 1), sizeof(double));
    if (!ga || !gr || !Ru || gram_dd(m, n, A, lda, ga) != 0) {
        free(ga);
        free(gr);
        free(Ru);
        return -2.0;
    }
    /* the upper triangle of R, zeros below */
    for (int64_t k = 0; k < n; ++k)
        for (int64_t i = 0; i <= k; ++i) Ru[IDX(i, k, n)] = R[IDX(i, k, ldr)];
    if (gram_dd(n, n, Ru, n, gr) != 0) {
        free(ga);
        free(gr);
        free(Ru);
        return -2.0;
    }
    csum_t num = {0.0, 0.0}, den = {0.0, 0.0};
    int64_t t = 0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = j; k < n; ++k, ++t) {
            dd_t d = dd_sub(gr[t], ga[t]);
            double v = d.hi + d.lo;
            csum_add(&num, (j == k ? 1.0 : 2.0) * v * v);    /* off-diagonal entries appear twice */
            if (j == k) {
                csum_add(&den, ga[t].hi);
                csum_add(&den, ga[t].lo);
            }
        }
    free(ga);
    free(gr);
    free(Ru);
    double dn = csum_value(&den);
    if (!(dn > 0.0)) return -1.0;
    return sqrt(csum_value(&num)) / dn;
}
