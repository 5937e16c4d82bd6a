// Context, errors, device memory and the selector class table.
#include <cstdlib>
#include <cstring>

#include "internal.h"

int xab_fail(xab_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

int xab_hip_check(xab_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return XAB_OK;
    if (e == hipErrorOutOfMemory) return xab_fail(ctx, XAB_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return xab_fail(ctx, XAB_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void *xab_dalloc(xab_ctx *ctx, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (ctx->alloc_fn) {
        p = ctx->alloc_fn(bytes, ctx->user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) ctx->live[p] = bytes;
    return p;
}

size_t xab_dbytes(const xab_ctx *ctx, const void *p) {
    if (!p) return 0;
    auto it = ctx->live.find(p);
    return it == ctx->live.end() ? 0 : it->second;
}

void xab_dfree(xab_ctx *ctx, void *p) {
    if (!p) return;
    ctx->live.erase(p);
    if (ctx->free_fn) ctx->free_fn(p, ctx->user);
    else (void)hipFree(p);
}

void *xab_scratch(xab_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->scratch_bytes) return ctx->scratch;
    // the old buffer may still be read by queued work on this stream
    if (ctx->scratch) {
        (void)hipStreamSynchronize(ctx->stream);
        xab_dfree(ctx, ctx->scratch);
    }
    size_t want = bytes + bytes / 4 + 4096;
    ctx->scratch = xab_dalloc(ctx, want);
    ctx->scratch_bytes = ctx->scratch ? want : 0;
    return ctx->scratch;
}

extern "C" {

int xab_init(xab_ctx **out, const xab_init_opts *opts) {
    if (!out) return XAB_E_NULL;
    *out = nullptr;
    xab_ctx *ctx = new xab_ctx();
    if (opts) {
        if ((opts->alloc == nullptr) != (opts->free == nullptr)) {
            delete ctx;
            return XAB_E_NULL;
        }
        ctx->alloc_fn = opts->alloc;
        ctx->free_fn = opts->free;
        ctx->user = opts->user;
        ctx->stream = (hipStream_t)opts->stream;
        if (opts->policy < XAB_TIME || opts->policy > XAB_ACCURACY) {
            delete ctx;
            return XAB_E_SHAPE;
        }
        ctx->policy = opts->policy;
    }
    int dev = (opts && opts->device >= 0) ? opts->device : -1;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) {
            delete ctx;
            return XAB_E_DEVICE;
        }
    } else if (hipSetDevice(dev) != hipSuccess) {
        delete ctx;
        return XAB_E_DEVICE;
    }
    ctx->device = dev;
    ctx->d_flag = (int *)xab_dalloc(ctx, 256);
    if (!ctx->d_flag) {
        delete ctx;
        return XAB_E_NOMEM;
    }
    const int ns = xab_noalloc_setup(ctx);
    if (ns != XAB_OK) {
        xab_dfree(ctx, ctx->d_flag);
        delete ctx;
        return ns;
    }
    const char *pol = getenv("XAB_POLICY");
    if (pol) {
        if (!strcmp(pol, "TIME")) ctx->policy = XAB_TIME;
        else if (!strcmp(pol, "STABLE")) ctx->policy = XAB_STABLE;
        else if (!strcmp(pol, "LEARNED")) ctx->policy = XAB_LEARNED;
        else if (!strcmp(pol, "MEMORY")) ctx->policy = XAB_MEMORY;
        else if (!strcmp(pol, "ACCURACY")) ctx->policy = XAB_ACCURACY;
    }
    *out = ctx;
    return XAB_OK;
}

void xab_finalize(xab_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    xab_dfree(ctx, ctx->scratch);
    xab_dfree(ctx, ctx->d_flag);
    xab_dfree(ctx, ctx->d_mlp);
    delete ctx;
}

int xab_set_stream(xab_ctx *ctx, void *stream) {
    if (!ctx) return XAB_E_NULL;
    ctx->stream = (hipStream_t)stream;
    return XAB_OK;
}

const char *xab_last_error(const xab_ctx *ctx) { return ctx ? ctx->err : "null context"; }

const char *xab_status_str(int s) {
    switch (s) {
        case XAB_OK: return "ok";
        case XAB_E_NULL: return "null pointer";
        case XAB_E_SHAPE: return "bad shape";
        case XAB_E_DTYPE: return "unsupported precision";
        case XAB_E_STRUCT: return "invalid CSR structure";
        case XAB_E_ALIAS: return "input and output overlap";
        case XAB_E_UNSUPPORTED: return "variant not applicable";
        case XAB_E_NOMEM: return "out of device memory";
        case XAB_E_DEVICE: return "device error";
        case XAB_E_ALIGN: return "matrix array not 16-byte aligned";
        case XAB_NOT_CONVERGED: return "not converged";
        case XAB_BREAKDOWN: return "breakdown";
        case XAB_TIME_LIMIT: return "time limit";
        default: return "unknown status";
    }
}

// The selector's action space.  General: row-split with 1, 8 or 64 lanes
// per row; nnz-split with 2048 or 8192 entries per workgroup; segmented scan
// with 4, 8, 16 or 32 entries per lane; column-blocked segmented scan with
// its entries per lane chosen from the matrix size; sliced ELLPACK with chunks of 64 rows sorted in
// windows of 1024.  Symmetric: atomic transpose (baseline) and
// zero-block-omitted reduction with 64- or 256-row blocks (tiles of about
// 8192 entries and at most 1024 rows).
int xab_class_params(int32_t k, xab_variant *v, xab_params *p) {
    if (!v || !p) return XAB_E_NULL;
    xab_params q{};
    q.lanes_per_row = 8;
    q.tile_nnz = 2048;
    q.j_per_lane = 8;
    q.col_block = 256;
    q.tile_rows = 2048;
    switch (k) {
        case 0: *v = XAB_ROW; q.lanes_per_row = 1; break;
        case 1: *v = XAB_ROW; q.lanes_per_row = 8; break;
        case 2: *v = XAB_ROW; q.lanes_per_row = 64; break;
        case 3: *v = XAB_NNZ; q.tile_nnz = 2048; break;
        case 4: *v = XAB_NNZ; q.tile_nnz = 8192; break;
        case 5: *v = XAB_BSS; q.j_per_lane = 4; break;
        case 6: *v = XAB_BSS; q.j_per_lane = 8; break;
        case 7: *v = XAB_BSS; q.j_per_lane = 16; break;
        case 8: *v = XAB_BSS; q.j_per_lane = 32; break;
        case 9: *v = XAB_SYM_ATOMIC; q.lanes_per_row = 8; break;
        case 10: *v = XAB_SYM_S3; q.col_block = 64; q.tile_nnz = 8192; q.tile_rows = 1024; break;
        case 11: *v = XAB_SYM_S3; q.col_block = 256; q.tile_nnz = 8192; q.tile_rows = 1024; break;
        case 12: *v = XAB_XCB; q.j_per_lane = 0; break;
        case 13: *v = XAB_SELL; q.tile_rows = 1024; break;
        case 14: *v = XAB_BCSR; break;
        default: return XAB_E_SHAPE;
    }
    *p = q;
    return XAB_OK;
}

}  // extern "C"
