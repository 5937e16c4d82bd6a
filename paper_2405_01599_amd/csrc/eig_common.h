// Pieces shared by the restarted Lanczos and Arnoldi drivers: workspace,
// the device recurrence step, the basis rotation kernel and the residual
// kernel.  Included by lanczos.hip and arnoldi.hip (each gets its own copy
// of these internal kernels).
#pragma once
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "blas.h"

namespace {

constexpr double kEta = 0.70710678118654752440;  // DGKS threshold 1/sqrt(2)
constexpr int kMaxM = 63;                         // basis vectors per cycle (slots of the fused dots)
constexpr int kRotNT = 256;
constexpr int kMaxNarrowEig = 8;  // accuracy policy: tenfold narrowings of the threshold at most

// out[:, c] = sum_{j < mm} V[:, j] * Y[j + c * mm] for c < k (column-major
// Y; mm <= 64, k <= 64).  One row per thread, grid-stride: the thread keeps
// its row's k outputs in registers (K >= k of them) and streams the row's mm
// basis entries, eight loads in flight (coalesced across the wave); Y, the
// same for every thread, is read with scalar loads, eight consecutive
// entries of a column at a time, straight into the fma operands.  Each
// output is one fma chain over j = 0, 1, ..., mm - 1; every basis entry is
// read from HBM once and every output written once.  (A workgroup per 64
// rows staging the basis in LDS took 330 us for 30 vectors to 20 on the
// 2,097,152-row stencil; this takes 200 us.)
template <int K>
__global__ __launch_bounds__(kRotNT) void k_rotate(const double *__restrict__ V, int64_t ldv, int mm,
                                                   const double *__restrict__ Y, int k, double *__restrict__ out,
                                                   int64_t ldo, int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * kRotNT + threadIdx.x; r < n; r += (int64_t)gridDim.x * kRotNT) {
        double acc[K];
#pragma unroll
        for (int t = 0; t < K; ++t) acc[t] = 0.0;
        int j = 0;
        for (; j + 8 <= mm; j += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)(j + u) * ldv + r];
#pragma unroll
            for (int t = 0; t < K; ++t)
                if (t < k) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[t] = fma(v[u], Y[t * mm + j + u], acc[t]);
                }
        }
        for (; j < mm; ++j) {
            const double v = V[(int64_t)j * ldv + r];
#pragma unroll
            for (int t = 0; t < K; ++t)
                if (t < k) acc[t] = fma(v, Y[t * mm + j], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < K; ++t)
            if (t < k) out[(int64_t)t * ldo + r] = acc[t];
    }
}

// part[block] = sum over its rows of (ax - c1 x1 - c2 x2)^2 (x2 may be null)
__global__ __launch_bounds__(kRotNT) void k_eig_resid(const double *__restrict__ ax, const double *__restrict__ x1,
                                                      double c1, const double *__restrict__ x2, double c2, int64_t n,
                                                      double *__restrict__ part) {
    __shared__ double sh[kRotNT];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRotNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRotNT) {
        double d = ax[i] - c1 * x1[i];
        if (x2) d -= c2 * x2[i];
        acc = fma(d, d, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRotNT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Workspace: two bases of m + 1 vectors (the restart rotates one into the
// other), w, the reduction partials, per-step coefficient slots (h1 and h2,
// m + 2 each: dots then the norm, and the gated norm) followed by the
// per-step DGKS gates, and the rotation's coefficient matrix.
struct Work {
    xab_ctx *ctx = nullptr;
    char *base = nullptr;
    double *V = nullptr, *V2 = nullptr, *w = nullptr, *part = nullptr, *coef = nullptr, *Y = nullptr;
    int *gate = nullptr;
    int64_t ldv = 0;
    int ld = 0;  // doubles per step slot
    double *host = nullptr;
    size_t host_bytes = 0;
    ~Work() {
        if (base) xab_dfree(ctx, base);
        if (host) (void)hipHostFree(host);
    }
};

int alloc_work(xab_ctx *ctx, Work &W, int64_t n, int m) {
    W.ctx = ctx;
    W.ldv = (n + 63) / 64 * 64;
    W.ld = 2 * (m + 2) + 1;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t basis = al(sizeof(double) * (size_t)(m + 1) * W.ldv);
    const size_t o_V2 = basis, o_w = o_V2 + basis, o_part = o_w + al(sizeof(double) * W.ldv);
    const size_t o_coef = o_part + al(sizeof(double) * xab::kRedBlocks * xab::kPartLd);
    const size_t coef_bytes = sizeof(double) * (size_t)W.ld * m;
    const size_t o_gate = o_coef + coef_bytes;  // read back with the coefficients in one copy
    const size_t o_Y = o_coef + al(coef_bytes + sizeof(int) * m);
    const size_t total = o_Y + al(sizeof(double) * (size_t)(kMaxM + 1) * (kMaxM + 1));
    W.base = (char *)xab_dalloc(ctx, total);
    if (!W.base) return xab_fail(ctx, XAB_E_NOMEM, "Lanczos workspace (%zu bytes)", total);
    W.V = (double *)W.base;
    W.V2 = (double *)(W.base + o_V2);
    W.w = (double *)(W.base + o_w);
    W.part = (double *)(W.base + o_part);
    W.coef = (double *)(W.base + o_coef);
    W.gate = (int *)(W.base + o_gate);
    W.Y = (double *)(W.base + o_Y);
    W.host_bytes = coef_bytes + sizeof(int) * m;
    if (hipHostMalloc((void **)&W.host, std::max(W.host_bytes, sizeof(double) * (size_t)(kMaxM + 1) * (kMaxM + 1)),
                      hipHostMallocDefault) != hipSuccess) {
        W.host = nullptr;
        return xab_fail(ctx, XAB_E_NOMEM, "pinned host buffer");
    }
    return XAB_OK;
}

// The MM ratio of eq. (1) over samples v[s-t .. s-1]: max / min.
double mm_ratio(const std::vector<double> &v, size_t s, size_t t) {
    double mx = v[s - t], mn = v[s - t];
    for (size_t z = s - t; z < s; ++z) {
        mx = std::max(mx, v[z]);
        mn = std::min(mn, v[z]);
    }
    return mx / mn;
}

int rotate(xab_ctx *ctx, const Work &W, int mm, const std::vector<double> &Ycm, int k, double *out, int64_t ldo,
           int64_t n) {
    if (mm > 64 || k > 64) return xab_fail(ctx, XAB_E_SHAPE, "rotation of %d vectors to %d", mm, k);
    memcpy(W.host, Ycm.data(), sizeof(double) * (size_t)mm * k);
    XAB_HIP(ctx, hipMemcpyAsync(W.Y, W.host, sizeof(double) * (size_t)mm * k, hipMemcpyHostToDevice, ctx->stream));
    // the smallest instance that holds k outputs per thread
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kRotNT - 1) / kRotNT, 4096))), b(kRotNT);
    hipStream_t st = ctx->stream;
    if (k <= 8) hipLaunchKernelGGL((k_rotate<8>), g, b, 0, st, W.V, W.ldv, mm, W.Y, k, out, ldo, n);
    else if (k <= 16) hipLaunchKernelGGL((k_rotate<16>), g, b, 0, st, W.V, W.ldv, mm, W.Y, k, out, ldo, n);
    else if (k <= 24) hipLaunchKernelGGL((k_rotate<24>), g, b, 0, st, W.V, W.ldv, mm, W.Y, k, out, ldo, n);
    else if (k <= 32) hipLaunchKernelGGL((k_rotate<32>), g, b, 0, st, W.V, W.ldv, mm, W.Y, k, out, ldo, n);
    else if (k <= 48) hipLaunchKernelGGL((k_rotate<48>), g, b, 0, st, W.V, W.ldv, mm, W.Y, k, out, ldo, n);
    else hipLaunchKernelGGL((k_rotate<64>), g, b, 0, st, W.V, W.ldv, mm, W.Y, k, out, ldo, n);
    XAB_LAUNCH_CHECK(ctx, "k_rotate");
    // the pinned buffer is reused by the next read-back: finish the copy first
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return XAB_OK;
}


// One step of the Arnoldi / Lanczos recurrence on the device: w = A v_j,
// then w is orthogonalised against v_0 .. v_j by classical Gram-Schmidt
// with the DGKS second pass and stored, normalised, as v_{j+1}.  Slot j
// receives h1 (pass-one dots, then ||w||^2), h2 (pass-two dots, then
// ||w'||^2), the gated ||w''||^2 and the gate; nothing is read back.
int recurrence_step(xab_ctx *ctx, const xab_plan *pl, Work &W, int j, int mc, int64_t n) {
    const int nb = xab::kRedBlocks;
    int s;
    double *V = W.V, *vj = V + (int64_t)j * W.ldv;
    double *h1 = W.coef + (size_t)j * W.ld, *h2 = h1 + (mc + 2), *sc = h2 + (mc + 2);
    int *gate = W.gate + j;
    if ((s = xab_spmv_dispatch(ctx, pl, vj, XAB_F64, W.w, XAB_F64, XAB_F64)) != XAB_OK) return s;
    if ((s = xab::mdot<double>(ctx, V, W.ldv, j + 1, W.w, n, W.part, nb, nullptr)) != XAB_OK) return s;
    if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, j + 2, h1, 0, nullptr)) != XAB_OK) return s;
    if ((s = xab::update_mdot<double>(ctx, V, j + 1, h1, V, j + 1, W.ldv, W.w, n, W.part, nb)) != XAB_OK) return s;
    if ((s = xab::reduce_parts_dgks(ctx, W.part, nb, xab::kPartLd, j + 2, h2, h1 + j + 1, kEta, gate)) != XAB_OK)
        return s;
    if ((s = xab::update_norm<double>(ctx, V, W.ldv, j + 1, h2, W.w, n, W.part, nb, gate)) != XAB_OK) return s;
    if ((s = xab::reduce_parts(ctx, W.part, nb, 1, 1, sc, 0, gate)) != XAB_OK) return s;
    return xab::scale_precond<double>(ctx, W.w, h2 + j + 1, V + (int64_t)(j + 1) * W.ldv, nullptr, nullptr, n, sc,
                                      gate);
}

// ||x|| for a device vector (synchronous)
int device_norm(xab_ctx *ctx, Work &W, const double *x, int64_t n, double *out) {
    const int nb = xab::kRedBlocks;
    int s;
    if ((s = xab::mdot<double>(ctx, nullptr, 0, 0, x, n, W.part, nb, nullptr)) != XAB_OK) return s;
    if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, 1, W.coef, 0, nullptr)) != XAB_OK) return s;
    double v = 0.0;
    XAB_HIP(ctx, hipMemcpyAsync(&v, W.coef, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *out = std::sqrt(v);
    return XAB_OK;
}

}  // namespace
