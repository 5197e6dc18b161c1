/* fig1_dot.c -- a C program that uses libsalt through its C ABI alone:
 * device memory and a stream from the HIP runtime, no Python, no torch.
 *
 *   fig1_dot N A B C D DOT
 *
 * reads N binary64 values from each of the files A, B and C, evaluates the
 * paper's Fig. 1 tree d = a + (b - c) (one fused pass, salt_eval) and the
 * dot product a . b (salt_dot), both on one stream, and writes d (N values)
 * to the file D and the dot (one value) to DOT. Exit status 0 on success;
 * otherwise a message names the failing call.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "salt.h"

static int hip_failed(hipError_t e, const char *what) {
    if (e == hipSuccess) return 0;
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
}

static int salt_failed(salt_status s, const char *what) {
    if (s == SALT_OK) return 0;
    fprintf(stderr, "%s: %s (%s)\n", what, salt_status_string(s), salt_last_error());
    return 1;
}

static int read_f64(const char *path, double *v, long long n) {
    FILE *f = fopen(path, "rb");
    if (!f) return 1;
    const size_t got = fread(v, sizeof(double), (size_t)n, f);
    fclose(f);
    return got != (size_t)n;
}

static int write_f64(const char *path, const double *v, long long n) {
    FILE *f = fopen(path, "wb");
    if (!f) return 1;
    const size_t put = fwrite(v, sizeof(double), (size_t)n, f);
    return (fclose(f) != 0) | (put != (size_t)n);
}

int main(int argc, char **argv) {
    if (argc != 7) {
        fprintf(stderr, "usage: %s N A B C D DOT\n", argv[0]);
        return 2;
    }
    const long long n = atoll(argv[1]);
    if (n < 1) {
        fprintf(stderr, "N must be at least 1\n");
        return 2;
    }
    const size_t bytes = (size_t)n * sizeof(double);
    double *host = (double *)malloc(4 * bytes);
    if (!host) return 1;
    double *a = host, *b = host + n, *c = host + 2 * n, *d = host + 3 * n;
    if (read_f64(argv[2], a, n) || read_f64(argv[3], b, n) || read_f64(argv[4], c, n)) {
        fprintf(stderr, "cannot read %lld values from each input\n", n);
        return 1;
    }

    const size_t ws_bytes = salt_reduce_workspace_bytes(n, SALT_F64);
    void *da = NULL, *db = NULL, *dc = NULL, *dd = NULL, *dres = NULL, *dws = NULL;
    hipStream_t s = NULL;
    double dot = 0.0;
    int bad = hip_failed(hipMalloc(&da, bytes), "hipMalloc") || hip_failed(hipMalloc(&db, bytes), "hipMalloc") ||
              hip_failed(hipMalloc(&dc, bytes), "hipMalloc") || hip_failed(hipMalloc(&dd, bytes), "hipMalloc") ||
              hip_failed(hipMalloc(&dres, sizeof(double)), "hipMalloc") ||
              hip_failed(hipMalloc(&dws, ws_bytes ? ws_bytes : 8), "hipMalloc") ||
              hip_failed(hipStreamCreate(&s), "hipStreamCreate");
    if (!bad)
        bad = hip_failed(hipMemcpyAsync(da, a, bytes, hipMemcpyHostToDevice, s), "copy a") ||
              hip_failed(hipMemcpyAsync(db, b, bytes, hipMemcpyHostToDevice, s), "copy b") ||
              hip_failed(hipMemcpyAsync(dc, c, bytes, hipMemcpyHostToDevice, s), "copy c");
    if (!bad) {
        /* d = a + (b - c): postfix LOAD 0, LOAD 1, LOAD 2, SUB, ADD */
        const uint32_t prog[5] = {SALT_TOKEN(SALT_OP_LOAD, 0), SALT_TOKEN(SALT_OP_LOAD, 1),
                                  SALT_TOKEN(SALT_OP_LOAD, 2), SALT_TOKEN(SALT_OP_SUB, 0),
                                  SALT_TOKEN(SALT_OP_ADD, 0)};
        const void *ops[3] = {da, db, dc};
        bad = salt_failed(salt_eval(prog, 5, ops, 3, NULL, 0, dd, n, SALT_F64, s), "salt_eval") ||
              salt_failed(salt_dot(n, da, db, dres, dws, ws_bytes, SALT_F64, s), "salt_dot");
    }
    if (!bad)
        bad = hip_failed(hipMemcpyAsync(d, dd, bytes, hipMemcpyDeviceToHost, s), "copy d") ||
              hip_failed(hipMemcpyAsync(&dot, dres, sizeof(double), hipMemcpyDeviceToHost, s), "copy dot") ||
              hip_failed(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (!bad && (write_f64(argv[5], d, n) || write_f64(argv[6], &dot, 1))) {
        fprintf(stderr, "cannot write the outputs\n");
        bad = 1;
    }
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dc);
    (void)hipFree(dd);
    (void)hipFree(dres);
    (void)hipFree(dws);
    free(host);
    return bad;
}
