// Matrix features for the learned selector: one device pass over rowptr and
// colind accumulating integer statistics (exact, order independent), then
// the 12 features formed on the host from them.
#include <cmath>

#include "internal.h"

namespace {

constexpr int kNT = 256;
constexpr int kLanesPerRow = 8;

// stats: [0] n, [1] nnz, [2] sum len^2, [3] max len, [4] max |i-j|,
//        [5] empty rows, [6] rows longer than 64, [7] sum |i-j|,
//        [8] entries in rows with len * n > 4 * nnz
__global__ __launch_bounds__(kNT) void k_stats(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                               int32_t n, int64_t nnz, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[7][kNT / xab::kWave];
    const int64_t row = ((int64_t)blockIdx.x * kNT + threadIdx.x) / kLanesPerRow;
    const int lane = threadIdx.x % kLanesPerRow;
    unsigned long long s2 = 0, mx = 0, bw = 0, empty = 0, long64 = 0, sd = 0, heavy = 0;
    if (row < n) {
        const int64_t k0 = rowptr[row], k1 = rowptr[row + 1];
        const int64_t l = k1 - k0;
        if (lane == 0) {
            s2 = (unsigned long long)(l * l);
            mx = (unsigned long long)l;
            empty = l == 0;
            long64 = l > 64;
            heavy = (l * (int64_t)n > 4 * nnz) ? (unsigned long long)l : 0ull;
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
        atomicAdd(&out[2], s2);
        atomicMax(&out[3], mx);
        atomicMax(&out[4], bw);
        atomicAdd(&out[5], empty);
        atomicAdd(&out[6], long64);
        atomicAdd(&out[7], sd);
        atomicAdd(&out[8], heavy);
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

int xab_matrix_stats(xab_ctx *ctx, xab_matrix *A) {
    if (A->have_stats) return XAB_OK;
    unsigned long long *d = (unsigned long long *)xab_scratch(ctx, 16 * sizeof(unsigned long long));
    if (!d) return xab_fail(ctx, XAB_E_NOMEM, "features scratch");
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, ctx->stream, d, 16);
    if (A->n > 0) {
        int64_t threads = (int64_t)A->n * kLanesPerRow;
        hipLaunchKernelGGL(k_stats, dim3((unsigned)((threads + kNT - 1) / kNT)), dim3(kNT), 0, ctx->stream, A->rowptr,
                           A->colind, A->n, A->nnz, d);
        XAB_LAUNCH_CHECK(ctx, "k_stats");
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
