// Matrix features for the learned selector: one device pass over rowptr and
// colind accumulating integer statistics (exact, order independent), then
// the 12 features formed on the host from them.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace {

constexpr int kNT = 256;
constexpr int kLanesPerRow = 8;

constexpr int kMaxGroups = 4096;

// stats: [0] n, [1] nnz, [2] sum len^2, [3] max len, [4] max |i-j|,
//        [5] empty rows, [6] rows longer than 64, [7] sum |i-j|,
//        [8] entries in rows with len * n > 4 * nnz
// Grid-stride over rows; each workgroup writes its 7 partials (indices 2..8)
// to its own slot and k_stats_reduce combines the slots (integer arithmetic,
// so the result does not depend on the order).
__global__ __launch_bounds__(kNT) void k_stats(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                               int32_t n, int64_t nnz, unsigned long long *__restrict__ part) {
    __shared__ unsigned long long sh[7][kNT / xab::kWave];
    const int lane = threadIdx.x % kLanesPerRow;
    unsigned long long s2 = 0, mx = 0, bw = 0, empty = 0, long64 = 0, sd = 0, heavy = 0;
    const int64_t stride = (int64_t)gridDim.x * (kNT / kLanesPerRow);
    for (int64_t row = ((int64_t)blockIdx.x * kNT + threadIdx.x) / kLanesPerRow; row < n; row += stride) {
        const int64_t k0 = rowptr[row], k1 = rowptr[row + 1];
        const int64_t l = k1 - k0;
        if (lane == 0) {
            s2 += (unsigned long long)(l * l);
            mx = (unsigned long long)l > mx ? (unsigned long long)l : mx;
            empty += l == 0;
            long64 += l > 64;
            heavy += (l * (int64_t)n > 4 * nnz) ? (unsigned long long)l : 0ull;
        }
        for (int64_t k = k0 + lane; k < k1; k += kLanesPerRow) {
            int64_t d = row - (int64_t)colind[k];
            unsigned long long ad = (unsigned long long)(d < 0 ? -d : d);
            sd += ad;
            bw = ad > bw ? ad : bw;
        }
    }
    // wave reductions (sums and maxima of unsigned 64-bit integers)
#pragma unroll
    for (int m = xab::kWave / 2; m > 0; m >>= 1) {
        s2 += __shfl_xor(s2, m);
        empty += __shfl_xor(empty, m);
        long64 += __shfl_xor(long64, m);
        sd += __shfl_xor(sd, m);
        heavy += __shfl_xor(heavy, m);
        unsigned long long a = __shfl_xor(mx, m), b = __shfl_xor(bw, m);
        mx = a > mx ? a : mx;
        bw = b > bw ? b : bw;
    }
    const int w = threadIdx.x / xab::kWave;
    if (threadIdx.x % xab::kWave == 0) {
        sh[0][w] = s2; sh[1][w] = mx; sh[2][w] = bw; sh[3][w] = empty;
        sh[4][w] = long64; sh[5][w] = sd; sh[6][w] = heavy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kNT / xab::kWave; ++i) {
            s2 += sh[0][i]; mx = sh[1][i] > mx ? sh[1][i] : mx; bw = sh[2][i] > bw ? sh[2][i] : bw;
            empty += sh[3][i]; long64 += sh[4][i]; sd += sh[5][i]; heavy += sh[6][i];
        }
        unsigned long long *o = part + (int64_t)blockIdx.x * 8;
        o[0] = s2; o[1] = mx; o[2] = bw; o[3] = empty; o[4] = long64; o[5] = sd; o[6] = heavy;
    }
}

// out[2..8] from the per-workgroup slots (one workgroup)
__global__ __launch_bounds__(kNT) void k_stats_reduce(const unsigned long long *__restrict__ part, int groups,
                                                      unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[kNT];
    for (int c = 0; c < 7; ++c) {
        const bool is_max = (c == 1 || c == 2);
        unsigned long long a = 0;
        for (int g = threadIdx.x; g < groups; g += kNT) {
            const unsigned long long v = part[(int64_t)g * 8 + c];
            a = is_max ? (v > a ? v : a) : a + v;
        }
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int m = kNT / 2; m > 0; m >>= 1) {
            if (threadIdx.x < m) {
                const unsigned long long b = sh[threadIdx.x + m];
                sh[threadIdx.x] = is_max ? (b > sh[threadIdx.x] ? b : sh[threadIdx.x]) : sh[threadIdx.x] + b;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) out[2 + c] = sh[0];
        __syncthreads();
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

int xab_matrix_stats(xab_ctx *ctx, xab_matrix *A) {
    if (A->have_stats) return XAB_OK;
    const int64_t threads = (int64_t)A->n * kLanesPerRow;
    const int groups = (int)std::min<int64_t>(std::max<int64_t>((threads + kNT - 1) / kNT, 1), kMaxGroups);
    unsigned long long *d =
        (unsigned long long *)xab_scratch(ctx, (16 + 8 * (size_t)groups) * sizeof(unsigned long long));
    if (!d) return xab_fail(ctx, XAB_E_NOMEM, "features scratch");
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, ctx->stream, d, 16);
    if (A->n > 0) {
        hipLaunchKernelGGL(k_stats, dim3((unsigned)groups), dim3(kNT), 0, ctx->stream, A->rowptr, A->colind, A->n,
                           A->nnz, d + 16);
        XAB_LAUNCH_CHECK(ctx, "k_stats");
        hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(kNT), 0, ctx->stream, d + 16, groups, d);
        XAB_LAUNCH_CHECK(ctx, "k_stats_reduce");
    }
    unsigned long long h[16];
    XAB_HIP(ctx, hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    A->stats[0] = A->n;
    A->stats[1] = A->nnz;
    for (int i = 2; i < 9; ++i) A->stats[i] = (int64_t)h[i];
    A->have_stats = true;
    return XAB_OK;
}

// The 12 features from the integer statistics (FP64 arithmetic, then FP32).
void xab_stats_to_features(const int64_t *st, int sym, float *f) {
    double dn = (double)st[0], dnnz = (double)st[1];
    double mean = dnnz / dn;
    double var = (double)st[2] / dn - mean * mean;
    if (var < 0.0) var = 0.0;
    double dmx = (double)(st[3] > 0 ? st[3] : 1);
    double v[12];
    v[0] = std::log2(dn > 1.0 ? dn : 1.0);
    v[1] = std::log2(dnnz > 1.0 ? dnnz : 1.0);
    v[2] = mean;
    v[3] = std::log2(1.0 + var);
    v[4] = std::log2(dmx);
    v[5] = std::log2(mean > 0.0 ? dmx / mean : 1.0);
    v[6] = (double)st[4] / dn;
    v[7] = sym ? 1.0 : 0.0;
    v[8] = (double)st[5] / dn;
    v[9] = (double)st[6] / dn;
    v[10] = st[1] > 0 ? (double)st[7] / dnnz / dn : 0.0;
    v[11] = st[1] > 0 ? (double)st[8] / dnnz : 0.0;
    for (int i = 0; i < 12; ++i) f[i] = (float)v[i];
}

extern "C" int xab_features(xab_ctx *ctx, const xab_matrix *Ac, float *h_out, int64_t *h_stats) {
    if (!ctx || !Ac || !h_out) return XAB_E_NULL;
    if (Ac->n == 0) return xab_fail(ctx, XAB_E_SHAPE, "features of an empty matrix");
    xab_matrix *A = const_cast<xab_matrix *>(Ac);  // statistics are cached on the handle
    int s = xab_matrix_stats(ctx, A);
    if (s != XAB_OK) return s;
    xab_stats_to_features(A->stats, A->sym() ? 1 : 0, h_out);
    if (h_stats)
        for (int i = 0; i < 9; ++i) h_stats[i] = A->stats[i];
    return XAB_OK;
}
