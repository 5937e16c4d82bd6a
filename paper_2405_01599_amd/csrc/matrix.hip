// CRS matrix handle and its structural validation (device passes).
#include "internal.h"

namespace {

constexpr int kBadRowptr0 = 1, kBadRowptrN = 2, kNonMonotone = 4, kRowptrRange = 8, kColRange = 16,
              kUpperEntry = 32;

__global__ void k_fill_int(int *p, int v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Pass 1: rowptr[0] = 0, rowptr[n] = nnz, monotone, inside [0, nnz].
__global__ void k_check_rowptr(const int32_t *rowptr, int32_t n, int64_t nnz, int *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int bad = 0;
    int64_t r = rowptr[i];
    if (i == 0 && r != 0) bad |= kBadRowptr0;
    if (i == n && r != nnz) bad |= kBadRowptrN;
    if (r < 0 || r > nnz) bad |= kRowptrRange;
    if (i < n && rowptr[i + 1] < r) bad |= kNonMonotone;
    if (bad) atomicOr(flag, bad);
}

// Pass 2 (only after pass 1 succeeded, so every row range is inside
// [0, nnz)): one wave per row checks 0 <= col < ncols and, for lower
// storage, col <= row.
__global__ void k_check_cols(const int32_t *rowptr, const int32_t *colind, int32_t n, int32_t ncols, int sym,
                             int *flag) {
    int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / xab::kWave;
    int lane = threadIdx.x % xab::kWave;
    if (row >= n) return;
    int bad = 0;
    for (int64_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += xab::kWave) {
        int32_t c = colind[k];
        if (c < 0 || c >= ncols) bad |= kColRange;
        if (sym && c > row) bad |= kUpperEntry;
    }
    if (bad) atomicOr(flag, bad);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

static int validate(xab_ctx *ctx, const xab_matrix *A) {
    int *flag = ctx->d_flag;
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, flag, 0, 1);
    int64_t nth = (int64_t)A->n + 1;
    hipLaunchKernelGGL(k_check_rowptr, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, ctx->stream,
                       A->rowptr, A->n, A->nnz, flag);
    XAB_LAUNCH_CHECK(ctx, "k_check_rowptr");
    int h = 0;
    XAB_HIP(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h) return xab_fail(ctx, XAB_E_STRUCT, "invalid rowptr (flags 0x%x)", h);
    if (A->n > 0 && A->nnz > 0) {
        int64_t threads = (int64_t)A->n * xab::kWave;
        hipLaunchKernelGGL(k_check_cols, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, ctx->stream,
                           A->rowptr, A->colind, A->n, A->ncols, A->sym() ? 1 : 0, flag);
        XAB_LAUNCH_CHECK(ctx, "k_check_cols");
        XAB_HIP(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (h & kUpperEntry) return xab_fail(ctx, XAB_E_STRUCT, "entry above the diagonal in lower storage");
        if (h) return xab_fail(ctx, XAB_E_STRUCT, "column index out of range (flags 0x%x)", h);
    }
    return XAB_OK;
}

extern "C" {

int xab_matrix_csr(xab_ctx *ctx, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *d_rowptr,
                   const int32_t *d_colind, const void *d_val, xab_dtype vt, uint32_t flags, xab_matrix **out) {
    if (!ctx || !out) return XAB_E_NULL;
    *out = nullptr;
    if (nrows < 0 || ncols < 0 || nnz < 0 || nnz >= (int64_t(1) << 31))
        return xab_fail(ctx, XAB_E_SHAPE, "bad sizes n=%d ncols=%d nnz=%lld", nrows, ncols, (long long)nnz);
    if (!d_rowptr || (nnz > 0 && (!d_colind || !d_val))) return xab_fail(ctx, XAB_E_NULL, "null matrix array");
    if (vt != XAB_F64 && vt != XAB_F32) return xab_fail(ctx, XAB_E_DTYPE, "value type %d", (int)vt);
    if ((flags & XAB_SYM_LOWER) && nrows != ncols)
        return xab_fail(ctx, XAB_E_SHAPE, "symmetric storage needs a square matrix");
    if (!aligned16(d_rowptr) || (nnz > 0 && (!aligned16(d_colind) || !aligned16(d_val))))
        return xab_fail(ctx, XAB_E_ALIGN, "matrix arrays must be 16-byte aligned");
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    xab_matrix *A = new xab_matrix();
    A->ctx = ctx;
    A->n = nrows;
    A->ncols = ncols;
    A->nnz = nnz;
    A->rowptr = d_rowptr;
    A->colind = d_colind;
    if (vt == XAB_F64) {
        A->val64 = (const double *)d_val;
        A->has64 = true;
    } else {
        A->val32 = (const float *)d_val;
        A->has32 = true;
    }
    A->flags = flags;
    if (!(flags & XAB_TRUST_INPUT)) {
        int s = validate(ctx, A);
        if (s != XAB_OK) {
            delete A;
            return s;
        }
    }
    *out = A;
    return XAB_OK;
}

int xab_matrix_add_values(xab_matrix *A, const void *d_val, xab_dtype vt) {
    if (!A) return XAB_E_NULL;
    if (A->nnz > 0 && !d_val) return xab_fail(A->ctx, XAB_E_NULL, "null values");
    if (A->nnz > 0 && !aligned16(d_val)) return xab_fail(A->ctx, XAB_E_ALIGN, "values must be 16-byte aligned");
    if (vt == XAB_F64) {
        A->val64 = (const double *)d_val;
        A->has64 = true;
    } else if (vt == XAB_F32) {
        A->val32 = (const float *)d_val;
        A->has32 = true;
    } else {
        return xab_fail(A->ctx, XAB_E_DTYPE, "value type %d", (int)vt);
    }
    return XAB_OK;
}

void xab_matrix_destroy(xab_matrix *A) {
    if (!A) return;
    (void)hipStreamSynchronize(A->ctx->stream);
    xab_dfree(A->ctx, A->diag64);
    xab_dfree(A->ctx, A->diag32);
    delete A;
}

}  // extern "C"
