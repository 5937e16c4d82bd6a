// SpMV that allocates nothing: the branchless segmented scan (XAB_BSS) on a
// CSR matrix given by its arrays, with its tile descriptors and carries in a
// fixed device buffer that this file owns (one copy per GPU, held until the
// process ends).  The kernels are the BSS plan's own (the split kernel of
// the plan set-up, the tile kernel and the carry fix-up), so the result is
// the one xab_spmv_csr gives with a BSS plan of the same entries per lane.
#include <mutex>

#include "spmv_launch.h"

namespace {

constexpr size_t kScratchBytes = (size_t)XAB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The device buffer.  Host code never passes this name to a kernel or a
// copy: it takes the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices];  // address of `scratch` on each device, set once

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// byte offsets of the six arrays for P tiles (the FP64 worst case of the
// accumulation type), each 256-byte aligned
struct Layout {
    size_t carry_val, tail_val, row_lo, tile_row, carry_row, tail_row, end;
    explicit Layout(int64_t P) {
        size_t o = 0;
        carry_val = o;
        o += up256(8 * (size_t)P);
        tail_val = o;
        o += up256(8 * (size_t)P);
        row_lo = o;
        o += up256(4 * (size_t)(P + 1));
        tile_row = o;
        o += up256(4 * (size_t)(P + 1));
        carry_row = o;
        o += up256(4 * (size_t)P);
        tail_row = o;
        o += up256(4 * (size_t)P);
        end = o;
    }
};

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

template <class VT, class XT, class YT, class AT>
int run(xab_ctx *ctx, const xab::BssArgs &a, const void *val, const void *x, void *y) {
    return xab::launch_bss_raw<VT, XT, YT, AT>(ctx, a, (const VT *)val, (const XT *)x, (YT *)y);
}

}  // namespace

// Looks up the buffer's address on the context's device (current when
// called), once per device.
int xab_noalloc_setup(xab_ctx *ctx) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return xab_fail(ctx, XAB_E_DEVICE, "device %d beyond the allocation-free buffer table", ctx->device);
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_addr[ctx->device]) return XAB_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return xab_hip_check(ctx, e, "address of the allocation-free buffer");
    if (!ptr) return xab_fail(ctx, XAB_E_DEVICE, "address of the allocation-free buffer is null");
    g_addr[ctx->device] = ptr;
    return XAB_OK;
}

extern "C" int xab_spmv_csr_noalloc(xab_ctx *ctx, int32_t nrows, int32_t ncols, int64_t nnz,
                                    const int32_t *d_rowptr, const int32_t *d_colind, const void *d_val,
                                    int32_t j_per_lane, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                                    xab_dtype acc) {
    if (!ctx) return XAB_E_NULL;
    if (nrows < 0 || ncols < 0 || nnz < 0 || nnz >= (int64_t(1) << 31))
        return xab_fail(ctx, XAB_E_SHAPE, "nrows %d, ncols %d, nnz %lld", nrows, ncols, (long long)nnz);
    const bool pow2 = j_per_lane > 0 && (j_per_lane & (j_per_lane - 1)) == 0;
    if (!pow2 || j_per_lane > 32)
        return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane must be a power of two in [1, 32]");
    if (nrows == 0) return XAB_OK;
    if (!d_rowptr || !d_y || (nnz > 0 && (!d_colind || !d_val)) || (ncols > 0 && !d_x))
        return xab_fail(ctx, XAB_E_NULL, "null array");
    if (((uintptr_t)d_colind | (uintptr_t)d_val) & 15)
        return xab_fail(ctx, XAB_E_ALIGN, "colind and values must be 16-byte aligned");
    const size_t xs = xt == XAB_F64 ? 8 : 4, ys = yt == XAB_F64 ? 8 : 4;
    if (overlaps(d_x, (size_t)ncols * xs, d_y, (size_t)nrows * ys))
        return xab_fail(ctx, XAB_E_ALIAS, "x and y overlap");
    const int64_t T = 256 * (int64_t)j_per_lane;
    const int64_t P = nnz > 0 ? (nnz + T - 1) / T : 1;
    if (P > XAB_NOALLOC_MAX_TILES)
        return xab_fail(ctx, XAB_E_SHAPE, "%lld tiles of %lld entries exceed the allocation-free limit of %d",
                        (long long)P, (long long)T, XAB_NOALLOC_MAX_TILES);
    const Layout L(P);
    if (L.end > kScratchBytes) return xab_fail(ctx, XAB_E_SHAPE, "allocation-free buffer too small");
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    unsigned char *base;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        base = (unsigned char *)(ctx->device >= 0 && ctx->device < kMaxDevices ? g_addr[ctx->device] : nullptr);
    }
    if (!base) return xab_fail(ctx, XAB_E_DEVICE, "allocation-free buffer not set up on device %d", ctx->device);
    using Run = int (*)(xab_ctx *, const xab::BssArgs &, const void *, const void *, void *);
    Run f = nullptr;
    if (xt == XAB_F64 && yt == XAB_F64 && acc == XAB_F64) f = run<double, double, double, double>;
    else if (xt == XAB_F32 && yt == XAB_F32 && acc == XAB_F32) f = run<float, float, float, float>;
    else if (xt == XAB_F32 && yt == XAB_F32 && acc == XAB_F64) f = run<float, float, float, double>;
    else if (xt == XAB_F32 && yt == XAB_F64 && acc == XAB_F64) f = run<float, float, double, double>;
    if (f) {
        const xab::BssArgs a{d_rowptr,
                             d_colind,
                             nnz,
                             P,
                             j_per_lane,
                             (const int32_t *)(base + L.row_lo),
                             (const int32_t *)(base + L.carry_row),
                             base + L.carry_val,
                             base + L.tail_val,
                             (int32_t *)(base + L.tail_row)};
        xab_launch_split_bss(ctx->stream, d_rowptr, nrows, T, P, (int32_t *)(base + L.row_lo),
                             (int32_t *)(base + L.tile_row), (int32_t *)(base + L.carry_row));
        XAB_LAUNCH_CHECK(ctx, "k_split_bss");
        return f(ctx, a, d_val, d_x, d_y);
    }
    return xab_fail(ctx, XAB_E_DTYPE, "unsupported (x, y, acc) = (%d, %d, %d)", (int)xt, (int)yt, (int)acc);
}
