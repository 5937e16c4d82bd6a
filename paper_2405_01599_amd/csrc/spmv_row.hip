// Row-based SpMV (the paper's conventional row decomposition) and the
// symmetric baseline whose transpose part is scattered with device atomics.
#include "spmv_launch.h"

namespace xab {
namespace {

constexpr int kNT = 256;

// S lanes per row, 256 / S rows per workgroup (equal rows, not equal work).
template <class VT, class XT, class YT, class AT, int S>
__global__ __launch_bounds__(kNT) void k_spmv_row(const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                                  const XT *__restrict__ x, YT *__restrict__ y, int32_t n,
                                                  int64_t nblocks) {
    constexpr int RPB = kNT / S;
    const int64_t blk = xcd_remap(blockIdx.x, nblocks);
    const int64_t row = blk * RPB + threadIdx.x / S;
    const int lane = threadIdx.x % S;
    AT acc = AT(0);
    if (row < n) {
        const int64_t k1 = rowptr[row + 1];
        for (int64_t k = rowptr[row] + lane; k < k1; k += S)
            acc += (AT)__builtin_nontemporal_load(val + k) * (AT)x[__builtin_nontemporal_load(colind + k)];
    }
#pragma unroll
    for (int m = S / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, S);
    if (row < n && lane == 0) y[row] = (YT)acc;
}

template <class T>
__global__ void k_zero(T *__restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = T(0);
}

// y must be zero on entry.  Each row adds its own sum and scatters
// L_ij x_i to y_j for its strictly lower entries, all by atomics.
template <class VT, class XT, class YT, int S>
__global__ __launch_bounds__(kNT) void k_spmv_sym_atomic(const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ colind,
                                                         const VT *__restrict__ val, const XT *__restrict__ x,
                                                         YT *__restrict__ y, int32_t n, int64_t nblocks) {
    constexpr int RPB = kNT / S;
    const int64_t blk = xcd_remap(blockIdx.x, nblocks);
    const int64_t row = blk * RPB + threadIdx.x / S;
    const int lane = threadIdx.x % S;
    YT acc = YT(0);
    if (row < n) {
        const YT xr = (YT)x[row];
        const int64_t k1 = rowptr[row + 1];
        for (int64_t k = rowptr[row] + lane; k < k1; k += S) {
            const int32_t j = colind[k];
            const YT v = (YT)val[k];
            acc += v * (YT)x[j];
            if (j < row) atomicAdd(&y[j], v * xr);
        }
    }
#pragma unroll
    for (int m = S / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, S);
    if (row < n && lane == 0) atomicAdd(&y[row], acc);
}

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <class VT, class XT, class YT, class AT, int S>
static int launch_row_s(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    hipLaunchKernelGGL((k_spmv_row<VT, XT, YT, AT, S>), dim3((unsigned)pl->P), dim3(kNT), 0, ctx->stream, A->rowptr,
                       A->colind, val, x, y, A->n, pl->P);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_row");
    return XAB_OK;
}

template <class VT, class XT, class YT, class AT>
int launch_row(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    switch (pl->params.lanes_per_row) {
        case 1: return launch_row_s<VT, XT, YT, AT, 1>(ctx, pl, val, x, y);
        case 2: return launch_row_s<VT, XT, YT, AT, 2>(ctx, pl, val, x, y);
        case 4: return launch_row_s<VT, XT, YT, AT, 4>(ctx, pl, val, x, y);
        case 8: return launch_row_s<VT, XT, YT, AT, 8>(ctx, pl, val, x, y);
        case 16: return launch_row_s<VT, XT, YT, AT, 16>(ctx, pl, val, x, y);
        case 32: return launch_row_s<VT, XT, YT, AT, 32>(ctx, pl, val, x, y);
        case 64: return launch_row_s<VT, XT, YT, AT, 64>(ctx, pl, val, x, y);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "lanes_per_row %d", pl->params.lanes_per_row);
    }
}

template <class VT, class XT, class YT, int S>
static int launch_atomic_s(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    hipLaunchKernelGGL((k_zero<YT>), dim3(grid_for(A->n, 256)), dim3(256), 0, ctx->stream, y, (int64_t)A->n);
    hipLaunchKernelGGL((k_spmv_sym_atomic<VT, XT, YT, S>), dim3((unsigned)pl->P), dim3(kNT), 0, ctx->stream,
                       A->rowptr, A->colind, val, x, y, A->n, pl->P);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_sym_atomic");
    return XAB_OK;
}

// The atomic baseline accumulates in the output type: it serves the
// combinations whose output and accumulation types agree.
template <class VT, class XT, class YT, class AT>
int launch_sym_atomic(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    if constexpr (!std::is_same<YT, AT>::value) {
        return xab_fail(ctx, XAB_E_DTYPE, "atomic symmetric SpMV needs output type == accumulation type");
    } else {
        switch (pl->params.lanes_per_row) {
            case 1: return launch_atomic_s<VT, XT, YT, 1>(ctx, pl, val, x, y);
            case 2: return launch_atomic_s<VT, XT, YT, 2>(ctx, pl, val, x, y);
            case 4: return launch_atomic_s<VT, XT, YT, 4>(ctx, pl, val, x, y);
            case 8: return launch_atomic_s<VT, XT, YT, 8>(ctx, pl, val, x, y);
            case 16: return launch_atomic_s<VT, XT, YT, 16>(ctx, pl, val, x, y);
            case 32: return launch_atomic_s<VT, XT, YT, 32>(ctx, pl, val, x, y);
            case 64: return launch_atomic_s<VT, XT, YT, 64>(ctx, pl, val, x, y);
            default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "lanes_per_row %d", pl->params.lanes_per_row);
        }
    }
}

XAB_INSTANTIATE_LAUNCHER(launch_row)
XAB_INSTANTIATE_LAUNCHER(launch_sym_atomic)

}  // namespace xab
