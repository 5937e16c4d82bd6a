// Host launchers of the SpMV kernels (one per implementation), explicitly
// instantiated for the supported precision combinations
// <values, x, y, accumulate>: <d,d,d,d>, <f,f,f,f>, <f,f,f,d>, <f,f,d,d>.
#pragma once
#include "internal.h"

namespace xab {
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
