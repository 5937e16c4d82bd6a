/* A plain C99 program that uses the library through include/xab.h alone:
 * it reads a CSR matrix, x and b from a file, moves them to the device,
 * selects an SpMV implementation (TIME), computes y = A x, solves A s = b
 * with GMRES(30) + Jacobi to 1e-10, and writes the results.  The GPU test
 * compares them with the oracle; built in-tree by __graft_entry__.build().
 *
 * Input  (little endian): int32 n, int64 nnz, int32 rowptr[n+1],
 *        int32 colind[nnz], f64 val[nnz], f64 x[n], f64 b[n].
 * Output: int32 chosen class, int32 spmv status, int32 gmres status,
 *        int64 iterations, f64 true relative residual, f64 y[n], f64 s[n].
 * Exit status 0 on success, 1 on a usage / file error, 2 on a library or
 * HIP error (its message on stderr). */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "xab.h"

static int rd(FILE *f, void *p, size_t sz, size_t cnt) { return fread(p, sz, cnt, f) == cnt; }

static void *to_device(const void *h, size_t bytes) {
    void *d = NULL;
    if (hipMalloc(&d, bytes ? bytes : 1) != hipSuccess) return NULL;
    if (bytes && hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return NULL;
    return d;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 1;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 1;
    int32_t n = 0;
    int64_t nnz = 0;
    if (!rd(f, &n, 4, 1) || !rd(f, &nnz, 8, 1) || n < 1 || nnz < 0) return 1;
    int32_t *rowptr = malloc(4 * (size_t)(n + 1)), *colind = malloc(4 * (size_t)(nnz ? nnz : 1));
    double *val = malloc(8 * (size_t)(nnz ? nnz : 1)), *x = malloc(8 * (size_t)n), *b = malloc(8 * (size_t)n);
    double *y = malloc(8 * (size_t)n), *s = malloc(8 * (size_t)n);
    if (!rowptr || !colind || !val || !x || !b || !y || !s) return 1;
    if (!rd(f, rowptr, 4, (size_t)n + 1) || !rd(f, colind, 4, (size_t)nnz) || !rd(f, val, 8, (size_t)nnz) ||
        !rd(f, x, 8, (size_t)n) || !rd(f, b, 8, (size_t)n))
        return 1;
    fclose(f);

    int32_t *d_rowptr = to_device(rowptr, 4 * (size_t)(n + 1));
    int32_t *d_colind = to_device(colind, 4 * (size_t)nnz);
    double *d_val = to_device(val, 8 * (size_t)nnz), *d_x = to_device(x, 8 * (size_t)n);
    double *d_b = to_device(b, 8 * (size_t)n), *d_y = NULL, *d_s = NULL;
    if (hipMalloc((void **)&d_y, 8 * (size_t)n) != hipSuccess || hipMalloc((void **)&d_s, 8 * (size_t)n) != hipSuccess ||
        hipMemset(d_s, 0, 8 * (size_t)n) != hipSuccess || !d_rowptr || !d_colind || !d_val || !d_x || !d_b) {
        fprintf(stderr, "device allocation failed\n");
        return 2;
    }

    xab_ctx *ctx = NULL;
    xab_matrix *A = NULL;
    xab_plan *plan = NULL;
    xab_select_info info;
    int st = xab_init(&ctx, NULL);
    if (st == XAB_OK) st = xab_matrix_csr(ctx, n, n, nnz, d_rowptr, d_colind, d_val, XAB_F64, 0, &A);
    if (st == XAB_OK) st = xab_select(ctx, A, XAB_TIME, &plan, &info);
    if (st != XAB_OK) {
        fprintf(stderr, "set-up: %s (%s)\n", xab_status_str(st), ctx ? xab_last_error(ctx) : "");
        return 2;
    }
    const int spmv = xab_spmv_csr(ctx, plan, d_x, XAB_F64, d_y, XAB_F64, XAB_F64);
    xab_krylov_opts o;
    memset(&o, 0, sizeof o);
    o.m = 30;
    o.tol = 1e-10;
    o.maxiter = 5000;
    o.mode = XAB_MODE_FP64;
    o.precond = XAB_PRECOND_JACOBI;
    o.m_max = 30;
    xab_krylov_info ki;
    memset(&ki, 0, sizeof ki);
    const int gm = xab_gmres(ctx, plan, d_b, d_s, &o, &ki);
    if (spmv < 0 || gm < 0) {
        fprintf(stderr, "compute: %s / %s (%s)\n", xab_status_str(spmv), xab_status_str(gm), xab_last_error(ctx));
        return 2;
    }
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(y, d_y, 8 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(s, d_s, 8 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
        return 2;
    xab_plan_destroy(plan);
    xab_matrix_destroy(A);
    xab_finalize(ctx);

    FILE *g = fopen(argv[2], "wb");
    if (!g) return 1;
    const int32_t hdr[3] = {info.chosen, spmv, gm};
    const int64_t it = ki.iters;
    const double rr = ki.true_relres;
    int ok = fwrite(hdr, 4, 3, g) == 3 && fwrite(&it, 8, 1, g) == 1 && fwrite(&rr, 8, 1, g) == 1 &&
             fwrite(y, 8, (size_t)n, g) == (size_t)n && fwrite(s, 8, (size_t)n, g) == (size_t)n;
    fclose(g);
    hipFree(d_rowptr);
    hipFree(d_colind);
    hipFree(d_val);
    hipFree(d_x);
    hipFree(d_b);
    hipFree(d_y);
    hipFree(d_s);
    free(rowptr);
    free(colind);
    free(val);
    free(x);
    free(b);
    free(y);
    free(s);
    return ok ? 0 : 1;
}
