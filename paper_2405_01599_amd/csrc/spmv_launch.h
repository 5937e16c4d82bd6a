// Host launchers of the SpMV kernels (one per implementation), explicitly
// instantiated for the supported precision combinations
// <values, x, y, accumulate>: <d,d,d,d>, <f,f,f,f>, <f,f,f,d>, <f,f,d,d>.
#pragma once
#include "internal.h"

namespace xab {
// Branchless segmented scan over the entry stream, described by its tile
// descriptors and carry workspace (a plan's, or caller-provided memory):
// P tiles of 256 * j entries; row_lo[P + 1], carry_row[P] from the split
// kernel; carry_val[P], tail_val[P] (accumulation type), tail_row[P] are
// written before they are read, so they need no clearing.
struct BssArgs {
    const int32_t *rowptr;
    const int32_t *colind;
    int64_t nnz;
    int64_t P;
    int32_t j;
    const int32_t *row_lo;
    const int32_t *carry_row;
    void *carry_val;
    void *tail_val;
    int32_t *tail_row;
};
template <class VT, class XT, class YT, class AT>
int launch_bss_raw(xab_ctx *ctx, const BssArgs &a, const VT *val, const XT *x, YT *y);

template <class VT, class XT, class YT, class AT>
int launch_row(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_nnz(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_bss(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_sym_s3(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_sym_atomic(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_xcb(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_sell(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
template <class VT, class XT, class YT, class AT>
int launch_bcsr(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y);
}  // namespace xab

#define XAB_INSTANTIATE_LAUNCHER(name)                                                               \
    template int name<double, double, double, double>(xab_ctx *, const xab_plan *, const double *,   \
                                                      const double *, double *);                     \
    template int name<float, float, float, float>(xab_ctx *, const xab_plan *, const float *,        \
                                                  const float *, float *);                           \
    template int name<float, float, float, double>(xab_ctx *, const xab_plan *, const float *,       \
                                                   const float *, float *);                          \
    template int name<float, float, double, double>(xab_ctx *, const xab_plan *, const float *,      \
                                                    const float *, double *);
