/*
 * c_client.c -- a plain C caller of libtsqr.so, with no Python in between.
 *
 * Reads an m-by-n column-major FP64 matrix from a binary file, computes its R
 * factor on the GPU through the C ABI (tsqr_create, tsqr_workspace_bytes,
 * tsqr_geqr_r_f64 on a stream of its own), and writes R (n-by-n, column-major)
 * to another binary file.  It also checks that an illegal argument is reported
 * before anything is launched.  Device memory comes from the HIP runtime, as a
 * C application would allocate it.
 *
 *     c_client A.bin m n R.bin        exit status 0 on success
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "tsqr.h"

static int fail(const char *what, int code)
{
    fprintf(stderr, "c_client: %s failed (%d)\n", what, code);
    return 1;
}

int main(int argc, char **argv)
{
    if (argc != 5) {
        fprintf(stderr, "usage: %s A.bin m n R.bin\n", argv[0]);
        return 2;
    }
    const int64_t m = atoll(argv[2]), n = atoll(argv[3]);
    if (m < 1 || n < 1 || n > TSQR_MAX_N) return fail("size check", -1);
    double *A = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *R = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!A || !R) return fail("host allocation", 0);
    FILE *f = fopen(argv[1], "rb");
    if (!f || fread(A, sizeof(double), (size_t)(m * n), f) != (size_t)(m * n)) return fail("reading A", 0);
    fclose(f);

    tsqr_handle_t h = NULL;
    int st = tsqr_create(&h, 0);
    if (st) return fail("tsqr_create", st);
    const int64_t ws_bytes = tsqr_workspace_bytes(h, m, n, TSQR_F64);
    if (ws_bytes <= 0) return fail("tsqr_workspace_bytes", (int)ws_bytes);

    double *dA = NULL, *dR = NULL;
    void *dws = NULL;
    hipStream_t s = NULL;
    if (hipMalloc((void **)&dA, sizeof(double) * (size_t)(m * n)) != hipSuccess ||
        hipMalloc((void **)&dR, sizeof(double) * (size_t)(n * n)) != hipSuccess ||
        hipMalloc(&dws, (size_t)ws_bytes) != hipSuccess || hipStreamCreate(&s) != hipSuccess)
        return fail("device allocation", 0);
    if (hipMemcpy(dA, A, sizeof(double) * (size_t)(m * n), hipMemcpyHostToDevice) != hipSuccess)
        return fail("copy to device", 0);

    /* an illegal leading dimension is argument 5, reported before any launch */
    st = tsqr_geqr_r_f64(h, m, n, dA, m - 1, dR, n, dws, ws_bytes, s);
    if (m > 1 && st != -5) return fail("argument check", st);

    st = tsqr_geqr_r_f64(h, m, n, dA, m, dR, n, dws, ws_bytes, s);
    if (st) return fail("tsqr_geqr_r_f64", st);
    if (hipStreamSynchronize(s) != hipSuccess) return fail("stream synchronize", 0);
    if (hipMemcpy(R, dR, sizeof(double) * (size_t)(n * n), hipMemcpyDeviceToHost) != hipSuccess)
        return fail("copy to host", 0);

    f = fopen(argv[4], "wb");
    if (!f || fwrite(R, sizeof(double), (size_t)(n * n), f) != (size_t)(n * n)) return fail("writing R", 0);
    fclose(f);

    (void)hipStreamDestroy(s);
    (void)hipFree(dA);
    (void)hipFree(dR);
    (void)hipFree(dws);
    tsqr_destroy(h);
    free(A);
    free(R);
    printf("c_client ok: m=%lld n=%lld\n", (long long)m, (long long)n);
    return 0;
}
