// Level-1 / Gram-Schmidt kernels of the Krylov drivers (host wrappers).
#pragma once
#include "internal.h"

namespace xab {

constexpr int kPartLd = 72;    // stride of one workgroup's partial sums (>= 64 vectors + norm)
constexpr int kRedBlocks = 2048; // workgroups of the reduction kernels (8 per CU)

template <class T>
int mdot(xab_ctx *ctx, const T *V, int64_t ldv, int nv, const T *w, int64_t n, double *part, int nb,
         const int *gate);
template <class T>
int update_norm(xab_ctx *ctx, const T *V, int64_t ldv, int nv, const double *h, T *w, int64_t n, double *part,
                int nb, const int *gate);
// w -= Vu h (nvu columns) and, in the same sweep, partials of Vd^T w (nvd
// columns, 0 for none) and ||w||^2 of the new w, in kPartLd slots per
// workgroup (the dots first, the norm at index nvd)
template <class T>
int update_mdot(xab_ctx *ctx, const T *Vu, int nvu, const double *h, const T *Vd, int nvd, int64_t ldv, T *w,
                int64_t n, double *part, int nb);
int reduce_parts(xab_ctx *ctx, const double *part, int nb, int ldp, int m, double *out, int add, const int *gate);
// reduce_parts (m slots, no accumulate) and, from its last slot (the
// squared norm after the first pass), the DGKS decision against *wn2
int reduce_parts_dgks(xab_ctx *ctx, const double *part, int nb, int ldp, int m, double *out, const double *wn2,
                      double eta, int *gate);

// row r of v = w / ||w||, z = M^-1 v, the squared norm being *nrm2_gated
// when a gate is given and set, else *nrm2
template <class T>
__device__ __forceinline__ void scale_precond_row(const T *__restrict__ w, const double *__restrict__ nrm2,
                                                  const double *__restrict__ nrm2_gated, const int *__restrict__ gate,
                                                  T *__restrict__ v, T *__restrict__ z, const T *__restrict__ d,
                                                  int64_t r) {
    const double s = sqrt((gate && *gate) ? *nrm2_gated : *nrm2);
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    const T vr = (T)((double)w[r] * inv);
    v[r] = vr;
    if (z) z[r] = d ? (T)((double)vr / (double)d[r]) : vr;
}
// v = w / ||w||, z = M^-1 v; the squared norm is *nrm2_gated when gate is
// non-null and set, else *nrm2
template <class T>
int scale_precond(xab_ctx *ctx, const T *w, const double *nrm2, T *v, T *z, const T *d, int64_t n,
                  const double *nrm2_gated = nullptr, const int *gate = nullptr);
template <class TS, class T>
int scale_from(xab_ctx *ctx, const TS *r, double scale, T *v, T *z, const T *d, int64_t n);
int residual(xab_ctx *ctx, const double *b, double *r, int64_t n, double *part, int nb);
template <class T>
int combine(xab_ctx *ctx, const T *V, int64_t ldv, int k, const double *y, double scale, const T *d, double *x,
            int64_t n);
template <class T>
int copy_cast(xab_ctx *ctx, const double *s, T *d, int64_t n);

__global__ void k_reduce_parts(const double *part, int nb, int ldp, int m, double *out, int add, const int *gate);

}  // namespace xab
