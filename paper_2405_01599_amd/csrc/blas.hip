// Level-1 kernels of the Krylov drivers.  Every reduction is two-stage and
// fixed-order (per-workgroup partials, then one ordered sum), so results do
// not depend on scheduling.  Basis vectors may be FP64 or FP32; inner
// products always accumulate in FP64.
#include "blas.h"

namespace xab {
namespace {

constexpr int kNT = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kNT / kWave; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Wave sum through DPP moves: the total lands in the last lane.
struct AddStep {
    template <int CTRL, int RM>
    __device__ __forceinline__ double apply(double s) const {
        return s + dpp_move<CTRL, RM>(s);
    }
};

// FP32 vectors are swept two consecutive rows per thread with 8-byte loads
// (every vector of the basis and the work vectors start on a 64-element
// boundary, so row pairs are 8-byte aligned); FP64 vectors one row per
// thread, the basis read with non-temporal loads (it streams through once
// per sweep, and the work vector then stays cached between the sweeps; the
// FP32 pairs are faster with ordinary loads).
template <class T>
constexpr int rows_per_thread() { return sizeof(T) == 4 ? 2 : 1; }
template <class T>
using Pair = T __attribute__((ext_vector_type(2)));

// part[b * ldp + i] = sum over this workgroup's rows of V_i[r] * w[r]
// (i < nv), part[b * ldp + nv] = sum of w[r]^2.  Rows are dealt in
// contiguous chunks of 256 to the workgroups.  The nv + 1 sums are reduced
// per wave with DPP (fixed order), then across the waves in wave order.
template <class T, int NV>
__device__ __forceinline__ void mdot_body(const T *__restrict__ V, int64_t ldv, int nv, const T *__restrict__ w,
                                          int64_t n, double *__restrict__ part, int ldp) {
    __shared__ double sh[kNT / kWave][NV + 1];
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    constexpr int R = rows_per_thread<T>();
    for (int64_t r = ((int64_t)blockIdx.x * kNT + threadIdx.x) * R; r < n; r += (int64_t)gridDim.x * kNT * R) {
        if (R == 2 && r + 1 < n) {
            // two rows: every load first (selects, no branches), then the products
            Pair<T> vp[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i)
                vp[i] = i < nv ? *reinterpret_cast<const Pair<T> *>(V + i * ldv + r) : Pair<T>(T(0));
            const Pair<T> wp = *reinterpret_cast<const Pair<T> *>(w + r);
            const double w0 = (double)wp[0], w1 = (double)wp[1];
            acc[NV] += w0 * w0;
            acc[NV] += w1 * w1;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                acc[i] += (double)vp[i][0] * w0;
                acc[i] += (double)vp[i][1] * w1;
            }
        } else {
            // one row: every load of the row first, then the products
            double vr[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) vr[i] = i < nv ? (double)ld_nt(V + i * ldv + r) : 0.0;
            const double wr = (double)w[r];
            acc[NV] += wr * wr;
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] += vr[i] * wr;
        }
    }
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
        const double t = wave_scan_dpp(acc[i], AddStep{});
        if (lane == kWave - 1) sh[wv][i] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x <= nv) {
        const int src = (int)threadIdx.x < nv ? (int)threadIdx.x : NV;
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kNT / kWave; ++q) t += sh[q][src];
        part[(int64_t)blockIdx.x * ldp + threadIdx.x] = t;
    }
}

template <class T, int NV>
__global__ __launch_bounds__(kNT) void k_mdot(const T *__restrict__ V, int64_t ldv, int nv, const T *__restrict__ w,
                                              int64_t n, double *__restrict__ part, int ldp) {
    mdot_body<T, NV>(V, ldv, nv, w, n, part, ldp);
}

// w -= sum_i h[i] V_i (i < nv); part[b] = sum of the new w^2.  When `gate`
// is given and *gate == 0 the kernel does nothing (the conditional second
// Gram-Schmidt pass was not needed).
template <class T, int NV>
__global__ __launch_bounds__(kNT) void k_update_norm(const T *__restrict__ V, int64_t ldv, int nv,
                                                     const double *__restrict__ h, T *__restrict__ w, int64_t n,
                                                     double *__restrict__ part, const int *__restrict__ gate) {
    __shared__ double sh[kNT / kWave];
    if (gate && *gate == 0) return;
    double hh[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hh[i] = i < nv ? h[i] : 0.0;
    double acc = 0.0;
    constexpr int R = rows_per_thread<T>();
    for (int64_t r = ((int64_t)blockIdx.x * kNT + threadIdx.x) * R; r < n; r += (int64_t)gridDim.x * kNT * R) {
        if (R == 2 && r + 1 < n) {
            Pair<T> vp[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i)
                vp[i] = i < nv ? *reinterpret_cast<const Pair<T> *>(V + i * ldv + r) : Pair<T>(T(0));
            const Pair<T> wp = *reinterpret_cast<const Pair<T> *>(w + r);
            double a0 = (double)wp[0], a1 = (double)wp[1];
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                a0 -= hh[i] * (double)vp[i][0];
                a1 -= hh[i] * (double)vp[i][1];
            }
            Pair<T> out;
            out[0] = (T)a0;
            out[1] = (T)a1;
            *reinterpret_cast<Pair<T> *>(w + r) = out;
            acc += (double)out[0] * (double)out[0];
            acc += (double)out[1] * (double)out[1];
        } else {
            double vr[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) vr[i] = i < nv ? (double)ld_nt(V + i * ldv + r) : 0.0;
            double a = (double)w[r];
#pragma unroll
            for (int i = 0; i < NV; ++i) a -= hh[i] * vr[i];
            const T at = (T)a;
            w[r] = at;
            acc += (double)at * (double)at;
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// w' = w - sum_{i < nvu} h[i] Vu_i, stored, and in the same sweep the dots
// of the next projection: part[b * ldp + i] = sum Vd_i[r] w'[r] (i < nvd),
// part[b * ldp + nvd] = sum w'[r]^2 (w' as stored).  One read of the basis
// serves an update and the following projection: DGKS passes Vd = Vu (the
// second pass's dots), MGS one column and the next, BCGS one block of four
// and the next.
template <class T, int NV>
__global__ __launch_bounds__(kNT) void k_update_mdot(const T *__restrict__ Vu, int nvu, const double *__restrict__ h,
                                                     const T *__restrict__ Vd, int nvd, int64_t ldv,
                                                     T *__restrict__ w, int64_t n, double *__restrict__ part,
                                                     int ldp) {
    __shared__ double sh[kNT / kWave][NV + 1];
    double hh[NV], acc[NV + 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hh[i] = i < nvu ? h[i] : 0.0;
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    const bool same = Vd == Vu && nvd == nvu;
    constexpr int R = rows_per_thread<T>();
    for (int64_t r = ((int64_t)blockIdx.x * kNT + threadIdx.x) * R; r < n; r += (int64_t)gridDim.x * kNT * R) {
        if (R == 2 && r + 1 < n) {
            Pair<T> vp[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i)
                vp[i] = i < nvu ? *reinterpret_cast<const Pair<T> *>(Vu + i * ldv + r) : Pair<T>(T(0));
            const Pair<T> wp = *reinterpret_cast<const Pair<T> *>(w + r);
            double a0 = (double)wp[0], a1 = (double)wp[1];
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                a0 -= hh[i] * (double)vp[i][0];
                a1 -= hh[i] * (double)vp[i][1];
            }
            Pair<T> out;
            out[0] = (T)a0;
            out[1] = (T)a1;
            *reinterpret_cast<Pair<T> *>(w + r) = out;
            const double d0 = (double)out[0], d1 = (double)out[1];
            acc[NV] += d0 * d0;
            acc[NV] += d1 * d1;
            if (same) {
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    acc[i] += (double)vp[i][0] * d0;
                    acc[i] += (double)vp[i][1] * d1;
                }
            } else {
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    if (i < nvd) {
                        const Pair<T> q = *reinterpret_cast<const Pair<T> *>(Vd + i * ldv + r);
                        acc[i] += (double)q[0] * d0;
                        acc[i] += (double)q[1] * d1;
                    }
            }
            continue;
        }
        double vr[NV];
        double a = (double)w[r];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            vr[i] = i < nvu ? (double)ld_nt(Vu + i * ldv + r) : 0.0;
            a -= hh[i] * vr[i];
        }
        const T at = (T)a;
        w[r] = at;
        const double ad = (double)at;
        acc[NV] += ad * ad;
        if (same) {
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] += vr[i] * ad;
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i < nvd) acc[i] += (double)Vd[i * ldv + r] * ad;
        }
    }
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
        const double t = wave_scan_dpp(acc[i], AddStep{});
        if (lane == kWave - 1) sh[wv][i] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x <= nvd) {
        const int src = (int)threadIdx.x < nvd ? (int)threadIdx.x : NV;
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kNT / kWave; ++q) t += sh[q][src];
        part[(int64_t)blockIdx.x * ldp + threadIdx.x] = t;
    }
}

// the gated launch of the second Gram-Schmidt pass
template <class T, int NV>
__global__ __launch_bounds__(kNT) void k_mdot_gated(const T *__restrict__ V, int64_t ldv, int nv,
                                                    const T *__restrict__ w, int64_t n, double *__restrict__ part,
                                                    int ldp, const int *__restrict__ gate) {
    if (*gate == 0) return;
    mdot_body<T, NV>(V, ldv, nv, w, n, part, ldp);
}

}  // namespace

// out[i] = sum over b of part[b * ldp + i], i < m, one workgroup per i:
// lane t sums slots t, t + 256, ... in ascending order, then a fixed LDS
// tree joins the lanes.  Optional accumulate: out[i] += ... when add != 0.
// When `gate` is non-null and *gate == 0 nothing happens.
// slot i of the partials summed over the nb workgroups (every thread of
// the block returns the sum)
__device__ __forceinline__ double reduce_slot(const double *__restrict__ part, int nb, int ldp, int i,
                                              double *sh) {
    // the thread's partials in ascending b, their loads issued 8 at a time
    double a = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * kNT < nb; b += 8 * kNT) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = part[(int64_t)(b + u * kNT) * ldp + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) a += t[u];
    }
    for (; b < nb; b += kNT) a += part[(int64_t)b * ldp + i];
    sh[threadIdx.x] = a;
    __syncthreads();
#pragma unroll
    for (int d = kNT / 2; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(kNT) void k_reduce_parts(const double *__restrict__ part, int nb, int ldp, int m,
                                                      double *__restrict__ out, int add,
                                                      const int *__restrict__ gate) {
    __shared__ double sh[kNT];
    if (gate && *gate == 0) return;
    const int i = blockIdx.x;
    const double t = reduce_slot(part, nb, ldp, i, sh);
    if (threadIdx.x == 0) out[i] = add ? out[i] + t : t;
}

// k_reduce_parts (no accumulate, no gate) whose last slot is the squared
// norm of w' after the first Gram-Schmidt pass: its workgroup also takes
// the DGKS decision against the squared norm of w before the pass
__global__ __launch_bounds__(kNT) void k_reduce_parts_dgks(const double *__restrict__ part, int nb, int ldp, int m,
                                                           double *__restrict__ out,
                                                           const double *__restrict__ wnorm2, double eta,
                                                           int *__restrict__ gate) {
    __shared__ double sh[kNT];
    const int i = blockIdx.x;
    const double t = reduce_slot(part, nb, ldp, i, sh);
    if (threadIdx.x == 0) {
        out[i] = t;
        if (i == m - 1) *gate = (sqrt(t) < eta * sqrt(*wnorm2)) ? 1 : 0;
    }
}

// v = w / sqrt(nrm2) (stored as T), z = v / d (Jacobi) or v, where nrm2 is
// *nrm2_gated when a gate is given and set, else *nrm2
template <class T>
__global__ void k_scale_precond(const T *__restrict__ w, const double *__restrict__ nrm2,
                                const double *__restrict__ nrm2_gated, const int *__restrict__ gate,
                                T *__restrict__ v, T *__restrict__ z, const T *__restrict__ d, int64_t n) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    scale_precond_row(w, nrm2, nrm2_gated, gate, v, z, d, r);
}

// v = r * scale (scale given on the host), z = v / d or v
template <class TS, class T>
__global__ void k_scale_from(const TS *__restrict__ r, double scale, T *__restrict__ v, T *__restrict__ z,
                             const T *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T vr = (T)((double)r[i] * scale);
    v[i] = vr;
    if (z) z[i] = d ? (T)((double)vr / (double)d[i]) : vr;
}

// r = b - r (in place over the product), part[b] = sum r^2
__global__ __launch_bounds__(kNT) void k_residual(const double *__restrict__ b, double *__restrict__ r, int64_t n,
                                                  double *__restrict__ part) {
    __shared__ double sh[kNT / kWave];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        double v = b[i] - r[i];
        r[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// x += scale * M^-1 sum_i y[i] V_i   (FP64 x, T basis, diag in FP64 or null)
template <class T>
__global__ void k_combine(const T *__restrict__ V, int64_t ldv, int k, const double *__restrict__ y, double scale,
                          const T *__restrict__ d, double *__restrict__ x, int64_t n) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double a = 0.0;
    for (int i = 0; i < k; ++i) a += y[i] * (double)ld_nt(V + i * ldv + r);
    a *= scale;
    if (d) a /= (double)d[r];
    x[r] += a;
}

// diagonal of A (sum of the entries with col == row); 1 where it is 0
template <class VT>
__global__ void k_diag(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                       const VT *__restrict__ val, int32_t n, VT *__restrict__ d) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    VT a = VT(0);
    for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
        if (colind[k] == r) a += val[k];
    d[r] = a != VT(0) ? a : VT(1);
}

template <class T>
__global__ void k_copy_cast(const double *__restrict__ s, T *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (T)s[i];
}

// ------------------------------------------------------------------ host wrappers
// Each sweep holds one register (pair) per basis vector per row, so the
// instance is the smallest of 4, 8, 12, ..., 32, 40, 48, 64 that covers the
// vectors in play: past about 28 vectors (FP32 pairs) the update-and-dots
// sweep drops to one wave per SIMD, and the unused slots of a larger
// instance still cost their predicated work.  Steps of 4 to 32 took the
// mixed-precision GMRES(30) on the lower-stored 27-point 128^3 stencil
// from 16.6 to 15.2 ms.
template <class T>
int mdot(xab_ctx *ctx, const T *V, int64_t ldv, int nv, const T *w, int64_t n, double *part, int nb,
         const int *gate) {
    dim3 g(nb), b(kNT);
    const int ldp = kPartLd;
#define XAB_MDOT_CASE(NVC)                                                                                       \
    if (nv <= NVC) {                                                                                             \
        if (gate) hipLaunchKernelGGL((k_mdot_gated<T, NVC>), g, b, 0, ctx->stream, V, ldv, nv, w, n, part, ldp, gate); \
        else hipLaunchKernelGGL((k_mdot<T, NVC>), g, b, 0, ctx->stream, V, ldv, nv, w, n, part, ldp);            \
        XAB_LAUNCH_CHECK(ctx, "k_mdot");                                                                         \
        return XAB_OK;                                                                                           \
    }
    XAB_MDOT_CASE(8)
    XAB_MDOT_CASE(12)
    XAB_MDOT_CASE(16)
    XAB_MDOT_CASE(20)
    XAB_MDOT_CASE(24)
    XAB_MDOT_CASE(28)
    XAB_MDOT_CASE(32)
    XAB_MDOT_CASE(40)
    XAB_MDOT_CASE(48)
    XAB_MDOT_CASE(64)
#undef XAB_MDOT_CASE
    return xab_fail(ctx, XAB_E_UNSUPPORTED, "more than 64 basis vectors");
}

template <class T>
int update_norm(xab_ctx *ctx, const T *V, int64_t ldv, int nv, const double *h, T *w, int64_t n, double *part,
                int nb, const int *gate) {
    dim3 g(nb), b(kNT);
#define XAB_UPD_CASE(NVC)                                                                                \
    if (nv <= NVC) {                                                                                     \
        hipLaunchKernelGGL((k_update_norm<T, NVC>), g, b, 0, ctx->stream, V, ldv, nv, h, w, n, part, gate); \
        XAB_LAUNCH_CHECK(ctx, "k_update_norm");                                                          \
        return XAB_OK;                                                                                   \
    }
    XAB_UPD_CASE(8)
    XAB_UPD_CASE(12)
    XAB_UPD_CASE(16)
    XAB_UPD_CASE(20)
    XAB_UPD_CASE(24)
    XAB_UPD_CASE(28)
    XAB_UPD_CASE(32)
    XAB_UPD_CASE(40)
    XAB_UPD_CASE(48)
    XAB_UPD_CASE(64)
#undef XAB_UPD_CASE
    return xab_fail(ctx, XAB_E_UNSUPPORTED, "more than 64 basis vectors");
}

template <class T>
int update_mdot(xab_ctx *ctx, const T *Vu, int nvu, const double *h, const T *Vd, int nvd, int64_t ldv, T *w,
                int64_t n, double *part, int nb) {
    dim3 g(nb), b(kNT);
    const int ldp = kPartLd;
    const int nv = nvu > nvd ? nvu : nvd;
#define XAB_UPM_CASE(NVC)                                                                                         \
    if (nv <= NVC) {                                                                                              \
        hipLaunchKernelGGL((k_update_mdot<T, NVC>), g, b, 0, ctx->stream, Vu, nvu, h, Vd, nvd, ldv, w, n, part, ldp); \
        XAB_LAUNCH_CHECK(ctx, "k_update_mdot");                                                                   \
        return XAB_OK;                                                                                            \
    }
    XAB_UPM_CASE(4)
    XAB_UPM_CASE(8)
    XAB_UPM_CASE(12)
    XAB_UPM_CASE(16)
    XAB_UPM_CASE(20)
    XAB_UPM_CASE(24)
    XAB_UPM_CASE(28)
    XAB_UPM_CASE(32)
    XAB_UPM_CASE(40)
    XAB_UPM_CASE(48)
    XAB_UPM_CASE(64)
#undef XAB_UPM_CASE
    return xab_fail(ctx, XAB_E_UNSUPPORTED, "more than 64 basis vectors");
}
template int update_mdot<double>(xab_ctx *, const double *, int, const double *, const double *, int, int64_t,
                                 double *, int64_t, double *, int);
template int update_mdot<float>(xab_ctx *, const float *, int, const double *, const float *, int, int64_t, float *,
                                int64_t, double *, int);

template int mdot<double>(xab_ctx *, const double *, int64_t, int, const double *, int64_t, double *, int, const int *);
template int mdot<float>(xab_ctx *, const float *, int64_t, int, const float *, int64_t, double *, int, const int *);
template int update_norm<double>(xab_ctx *, const double *, int64_t, int, const double *, double *, int64_t, double *,
                                 int, const int *);
template int update_norm<float>(xab_ctx *, const float *, int64_t, int, const double *, float *, int64_t, double *,
                                int, const int *);

int reduce_parts(xab_ctx *ctx, const double *part, int nb, int ldp, int m, double *out, int add, const int *gate) {
    if (m <= 0) return XAB_OK;
    hipLaunchKernelGGL(k_reduce_parts, dim3(m), dim3(kNT), 0, ctx->stream, part, nb, ldp, m, out, add, gate);
    XAB_LAUNCH_CHECK(ctx, "k_reduce_parts");
    return XAB_OK;
}

int reduce_parts_dgks(xab_ctx *ctx, const double *part, int nb, int ldp, int m, double *out, const double *wn2,
                      double eta, int *gate) {
    if (m <= 0) return XAB_OK;
    hipLaunchKernelGGL(k_reduce_parts_dgks, dim3(m), dim3(kNT), 0, ctx->stream, part, nb, ldp, m, out, wn2, eta, gate);
    XAB_LAUNCH_CHECK(ctx, "k_reduce_parts_dgks");
    return XAB_OK;
}

template <class T>
int scale_precond(xab_ctx *ctx, const T *w, const double *nrm2, T *v, T *z, const T *d, int64_t n,
                  const double *nrm2_gated, const int *gate) {
    hipLaunchKernelGGL((k_scale_precond<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, w, nrm2,
                       nrm2_gated, gate, v, z, d, n);
    XAB_LAUNCH_CHECK(ctx, "k_scale_precond");
    return XAB_OK;
}
template int scale_precond<double>(xab_ctx *, const double *, const double *, double *, double *, const double *,
                                   int64_t, const double *, const int *);
template int scale_precond<float>(xab_ctx *, const float *, const double *, float *, float *, const float *, int64_t,
                                  const double *, const int *);

template <class TS, class T>
int scale_from(xab_ctx *ctx, const TS *r, double scale, T *v, T *z, const T *d, int64_t n) {
    hipLaunchKernelGGL((k_scale_from<TS, T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, r, scale, v,
                       z, d, n);
    XAB_LAUNCH_CHECK(ctx, "k_scale_from");
    return XAB_OK;
}
template int scale_from<double, double>(xab_ctx *, const double *, double, double *, double *, const double *, int64_t);
template int scale_from<double, float>(xab_ctx *, const double *, double, float *, float *, const float *, int64_t);

int residual(xab_ctx *ctx, const double *b, double *r, int64_t n, double *part, int nb) {
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(kNT), 0, ctx->stream, b, r, n, part);
    XAB_LAUNCH_CHECK(ctx, "k_residual");
    return XAB_OK;
}

template <class T>
int combine(xab_ctx *ctx, const T *V, int64_t ldv, int k, const double *y, double scale, const T *d, double *x,
            int64_t n) {
    hipLaunchKernelGGL((k_combine<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, V, ldv, k, y, scale,
                       d, x, n);
    XAB_LAUNCH_CHECK(ctx, "k_combine");
    return XAB_OK;
}
template int combine<double>(xab_ctx *, const double *, int64_t, int, const double *, double, const double *, double *,
                             int64_t);
template int combine<float>(xab_ctx *, const float *, int64_t, int, const double *, double, const float *, double *,
                            int64_t);

template <class T>
int copy_cast(xab_ctx *ctx, const double *s, T *d, int64_t n) {
    hipLaunchKernelGGL((k_copy_cast<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, s, d, n);
    XAB_LAUNCH_CHECK(ctx, "k_copy_cast");
    return XAB_OK;
}
template int copy_cast<float>(xab_ctx *, const double *, float *, int64_t);

}  // namespace xab

// Jacobi diagonal of A in every precision A holds (library-owned, cached)
int xab_matrix_diag(xab_ctx *ctx, xab_matrix *A) {
    unsigned g = (unsigned)((A->n + 255) / 256);
    if (A->n == 0) return XAB_OK;
    if (A->has64 && !A->diag64) {
        A->diag64 = (double *)xab_dalloc(ctx, sizeof(double) * A->n);
        if (!A->diag64) return xab_fail(ctx, XAB_E_NOMEM, "diagonal");
        hipLaunchKernelGGL((xab::k_diag<double>), dim3(g), dim3(256), 0, ctx->stream, A->rowptr, A->colind, A->val64,
                           A->n, A->diag64);
        XAB_LAUNCH_CHECK(ctx, "k_diag");
    }
    if (A->has32 && !A->diag32) {
        A->diag32 = (float *)xab_dalloc(ctx, sizeof(float) * A->n);
        if (!A->diag32) return xab_fail(ctx, XAB_E_NOMEM, "diagonal");
        hipLaunchKernelGGL((xab::k_diag<float>), dim3(g), dim3(256), 0, ctx->stream, A->rowptr, A->colind, A->val32,
                           A->n, A->diag32);
        XAB_LAUNCH_CHECK(ctx, "k_diag");
    }
    return XAB_OK;
}
