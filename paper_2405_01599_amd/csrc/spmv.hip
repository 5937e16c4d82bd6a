// SpMV entry points: argument checks and dispatch on (variant, precision).
#include <type_traits>

#include "spmv_launch.h"

namespace {

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

template <class VT, class XT, class YT, class AT>
int run(xab_ctx *ctx, const xab_plan *pl, const VT *val, const void *x, void *y) {
    const XT *xx = (const XT *)x;
    YT *yy = (YT *)y;
    switch (pl->variant) {
        case XAB_ROW: return xab::launch_row<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_NNZ: return xab::launch_nnz<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_BSS: return xab::launch_bss<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_SYM_S3: return xab::launch_sym_s3<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_SYM_ATOMIC: return xab::launch_sym_atomic<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_XCB: return xab::launch_xcb<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_SELL: return xab::launch_sell<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
        case XAB_BCSR: return xab::launch_bcsr<VT, XT, YT, AT>(ctx, pl, val, xx, yy);
    }
    return xab_fail(ctx, XAB_E_UNSUPPORTED, "variant %d", (int)pl->variant);
}

size_t dsize(xab_dtype t) { return t == XAB_F64 ? 8 : 4; }

}  // namespace

int xab_spmv_dispatch(xab_ctx *ctx, const xab_plan *pl, const void *x, xab_dtype xt, void *y, xab_dtype yt,
                      xab_dtype acc) {
    const xab_matrix *A = pl->A;
    if (A->n == 0) return XAB_OK;
    if ((A->ncols > 0 && !x) || !y) return xab_fail(ctx, XAB_E_NULL, "null x or y");
    if (overlaps(x, (size_t)A->ncols * dsize(xt), y, (size_t)A->n * dsize(yt)))
        return xab_fail(ctx, XAB_E_ALIAS, "x and y overlap");
    if (xt == XAB_F64 && yt == XAB_F64 && acc == XAB_F64) {
        if (!A->has64) return xab_fail(ctx, XAB_E_DTYPE, "matrix holds no FP64 values");
        return run<double, double, double, double>(ctx, pl, A->val64, x, y);
    }
    if (xt == XAB_F32) {
        if (!A->has32) return xab_fail(ctx, XAB_E_DTYPE, "matrix holds no FP32 values");
        if (yt == XAB_F32 && acc == XAB_F32) return run<float, float, float, float>(ctx, pl, A->val32, x, y);
        if (yt == XAB_F32 && acc == XAB_F64) return run<float, float, float, double>(ctx, pl, A->val32, x, y);
        if (yt == XAB_F64 && acc == XAB_F64) return run<float, float, double, double>(ctx, pl, A->val32, x, y);
    }
    return xab_fail(ctx, XAB_E_DTYPE, "unsupported (x, y, acc) = (%d, %d, %d)", (int)xt, (int)yt, (int)acc);
}

extern "C" {

int xab_spmv_csr(xab_ctx *ctx, const xab_plan *plan, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                 xab_dtype acc) {
    if (!ctx || !plan) return XAB_E_NULL;
    if (plan->A->sym()) return xab_fail(ctx, XAB_E_UNSUPPORTED, "xab_spmv_csr on a symmetric matrix");
    return xab_spmv_dispatch(ctx, plan, d_x, xt, d_y, yt, acc);
}

int xab_spmv_sym(xab_ctx *ctx, const xab_plan *plan, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                 xab_dtype acc) {
    if (!ctx || !plan) return XAB_E_NULL;
    if (!plan->A->sym()) return xab_fail(ctx, XAB_E_UNSUPPORTED, "xab_spmv_sym needs XAB_SYM_LOWER");
    return xab_spmv_dispatch(ctx, plan, d_x, xt, d_y, yt, acc);
}

int xab_time_spmv(xab_ctx *ctx, const xab_plan *plan, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                  xab_dtype acc, int32_t warmup, int32_t reps, float *ms) {
    if (!ctx || !plan || !ms) return XAB_E_NULL;
    if (reps < 1 || warmup < 0) return xab_fail(ctx, XAB_E_SHAPE, "reps must be >= 1");
    for (int i = 0; i < warmup; ++i) {
        int s = xab_spmv_dispatch(ctx, plan, d_x, xt, d_y, yt, acc);
        if (s != XAB_OK) return s;
    }
    hipEvent_t e0, e1;
    XAB_HIP(ctx, hipEventCreate(&e0));
    XAB_HIP(ctx, hipEventCreate(&e1));
    int s = XAB_OK;
    (void)hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < reps && s == XAB_OK; ++i) s = xab_spmv_dispatch(ctx, plan, d_x, xt, d_y, yt, acc);
    (void)hipEventRecord(e1, ctx->stream);
    hipError_t e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != XAB_OK) return s;
    if (e != hipSuccess) return xab_hip_check(ctx, e, "spmv timing");
    *ms = t / reps;
    return XAB_OK;
}

}  // extern "C"
