// Block CSR SpMV with 4 x 4 blocks: a group of 16 lanes takes one block
// row (rows 4R .. 4R+3), lane e = 4 i + j holding position (i, j) of every
// block, so the group reads each block's 16 row-major values as one
// contiguous run and a wave reads four such runs per load.  Lane e
// accumulates v * x[4 c + j] over the block row's blocks in ascending block
// column order; the four lanes of row i are then added in a fixed order
// ((j0 + j1) + (j2 + j3)).  Positions without a stored entry are skipped by
// a select on the block's mask, so a non-finite x entry never reaches
// another row.
#include "spmv_launch.h"

namespace xab {
namespace {

constexpr int kNT = 256;
constexpr int kB = xab_plan::kBcsrB;
constexpr int kLanes = kB * kB;              // lanes per block row
constexpr int kRowsPerWg = kNT / kLanes;     // block rows per workgroup
constexpr int kUnroll = 4;

template <class VT, class XT, class YT, class AT>
__global__ __launch_bounds__(kNT) void k_spmv_bcsr(const int32_t *__restrict__ brp, const int32_t *__restrict__ bci,
                                                   const int32_t *__restrict__ mask, const VT *__restrict__ bv,
                                                   const XT *__restrict__ x, YT *__restrict__ y, int32_t n,
                                                   int32_t ncols, int64_t nbr, int64_t nwg) {
    const int64_t R = xcd_remap(blockIdx.x, nwg) * kRowsPerWg + threadIdx.x / kLanes;
    const int e = threadIdx.x % kLanes, i = e / kB, j = e % kB;
    AT acc = AT(0);
    if (R < nbr) {
        const int32_t q1 = brp[R + 1];
        int32_t q = brp[R];
        // kUnroll blocks per step: all their loads issued before the products
        for (; q + kUnroll <= q1; q += kUnroll) {
            VT v[kUnroll];
            int32_t c[kUnroll], m[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                v[u] = __builtin_nontemporal_load(bv + (int64_t)(q + u) * kLanes + e);
                c[u] = bci[q + u] * kB + j;
                m[u] = mask[q + u];
            }
            AT xv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) xv[u] = c[u] < ncols ? (AT)x[c[u]] : AT(0);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const AT p = (AT)v[u] * xv[u];
                acc = (m[u] >> e) & 1 ? acc + p : acc;
            }
        }
        for (; q < q1; ++q) {
            const VT v = __builtin_nontemporal_load(bv + (int64_t)q * kLanes + e);
            const int32_t c = bci[q] * kB + j;
            const AT xv = c < ncols ? (AT)x[c] : AT(0);
            const AT p = (AT)v * xv;
            acc = (mask[q] >> e) & 1 ? acc + p : acc;
        }
    }
    // row i: (j0 + j1) + (j2 + j3), all lanes of the wave taking part
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    if (R < nbr && j == 0 && R * kB + i < n) y[R * kB + i] = (YT)acc;
}

}  // namespace

template <class VT, class XT, class YT, class AT>
int launch_bcsr(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    (void)val;  // the plan holds its own blocked copy of the values
    const VT *bv;
    if constexpr (sizeof(VT) == 8) bv = (const VT *)pl->bcsr_val64;
    else bv = (const VT *)pl->bcsr_val32;
    if (!bv) return xab_fail(ctx, XAB_E_DTYPE, "BCSR plan holds no values of this precision");
    if (pl->A->n == 0) return XAB_OK;
    const int64_t nwg = (pl->bcsr_nbr + kRowsPerWg - 1) / kRowsPerWg;
    hipLaunchKernelGGL((k_spmv_bcsr<VT, XT, YT, AT>), dim3((unsigned)nwg), dim3(kNT), 0, ctx->stream, pl->bcsr_brp,
                       pl->bcsr_bci, pl->bcsr_mask, bv, x, y, pl->A->n, pl->A->ncols, pl->bcsr_nbr, nwg);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_bcsr");
    return XAB_OK;
}

XAB_INSTANTIATE_LAUNCHER(launch_bcsr)

}  // namespace xab
