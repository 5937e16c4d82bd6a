// Sliced ELLPACK SpMV (SELL-C-sigma with C = 64, one wave per chunk): lane
// l of chunk c sums ordered row c * 64 + l over the chunk's columns,
// k = 0 .. width - 1, reading entry k of all 64 rows as one contiguous run
// (column-major chunk), and writes y[perm[row]].  Entries past a row's
// length are padding and are skipped by a select, so a non-finite x entry
// never reaches another row.  Rows are summed in order, one lane each
// (sell_body.h).
#include "sell_body.h"
#include "spmv_launch.h"

namespace xab {
namespace {

constexpr int kNT = 256;                 // 4 chunks per workgroup
constexpr int kC = xab_plan::kSellC;
constexpr int kUnroll = 4;

template <class VT, class XT, class YT, class AT>
__global__ __launch_bounds__(kNT) void k_spmv_sell(const int64_t *__restrict__ cptr, const int32_t *__restrict__ clen,
                                                   const int32_t *__restrict__ rlen, const int32_t *__restrict__ perm,
                                                   const int32_t *__restrict__ cols, const VT *__restrict__ val,
                                                   const XT *__restrict__ x, YT *__restrict__ y, int32_t n,
                                                   int64_t nch, int64_t nwg) {
    const int64_t wg = xcd_remap(blockIdx.x, nwg);
    const int64_t c = wg * (kNT / kC) + threadIdx.x / kC;
    if (c >= nch) return;
    const int l = threadIdx.x % kC;
    const int64_t r = c * kC + l;
    const int32_t len = rlen[r];  // 0 for the slots past n
    const AT acc = sell_lane_sum<VT, XT, AT, kUnroll>(val, cols, x, cptr[c] + l, clen[c], len);
    if (r < n) y[perm[r]] = (YT)acc;
}

}  // namespace

template <class VT, class XT, class YT, class AT>
int launch_sell(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    (void)val;  // the plan holds its own padded copy of the values
    const xab_sell &S = pl->sell;
    const VT *pv;
    if constexpr (sizeof(VT) == 8) pv = (const VT *)S.val64;
    else pv = (const VT *)S.val32;
    if (!pv) return xab_fail(ctx, XAB_E_DTYPE, "SELL plan holds no values of this precision");
    if (pl->A->n == 0) return XAB_OK;
    const int64_t nwg = (S.nch + kNT / kC - 1) / (kNT / kC);
    hipLaunchKernelGGL((k_spmv_sell<VT, XT, YT, AT>), dim3((unsigned)nwg), dim3(kNT), 0, ctx->stream, S.cptr, S.clen,
                       S.rlen, S.perm, S.cols, pv, x, y, pl->A->n, S.nch, nwg);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_sell");
    return XAB_OK;
}

XAB_INSTANTIATE_LAUNCHER(launch_sell)

}  // namespace xab
