// Learned selector: a 12-64-64-K FP32 MLP predicting log2(t_k / t_best) for
// every selector class, with hand-written forward, backward and Adam
// kernels, trained on the GPU.  Gradients are reduced in two fixed-order
// stages (per-workgroup partial sums, then a sum over workgroups), so a
// training run is bitwise reproducible.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace {

constexpr int F = 12, H = 64, K = XAB_NCLASSES;
constexpr int NP = XAB_MLP_NPARAMS;
constexpr int OW1 = 0, OB1 = OW1 + H * F, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + K * H;
static_assert(OB3 + K == NP, "parameter layout");
constexpr int kNT = 256;
constexpr int kSB = 32;  // samples per workgroup

// Forward for samples [s0, s0 + ns) held in LDS; fills z1, z2 (pre-ReLU)
// and o.  Thread t computes outputs t, t + 256, ... of each layer.
__device__ void forward_block(const float *p, const float *f, int ns, float *z1, float *z2, float *o) {
    const int tid = threadIdx.x;
    for (int q = tid; q < ns * H; q += kNT) {
        int s = q / H, i = q % H;
        float a = p[OB1 + i];
        for (int j = 0; j < F; ++j) a += p[OW1 + i * F + j] * f[s * F + j];
        z1[s * H + i] = a;
    }
    __syncthreads();
    for (int q = tid; q < ns * H; q += kNT) {
        int s = q / H, i = q % H;
        float a = p[OB2 + i];
        for (int j = 0; j < H; ++j) a += p[OW2 + i * H + j] * fmaxf(z1[s * H + j], 0.f);
        z2[s * H + i] = a;
    }
    __syncthreads();
    for (int q = tid; q < ns * K; q += kNT) {
        int s = q / K, k = q % K;
        float a = p[OB3 + k];
        for (int j = 0; j < H; ++j) a += p[OW3 + k * H + j] * fmaxf(z2[s * H + j], 0.f);
        o[s * K + k] = a;
    }
    __syncthreads();
}

__device__ void load_params(const float *__restrict__ gp, float *p) {
    for (int i = threadIdx.x; i < NP; i += kNT) p[i] = gp[i];
}

// features of sample idx(s) (optionally standardised) into LDS
__device__ void load_features(const float *__restrict__ feat, const int32_t *__restrict__ order, int64_t s0, int ns,
                              const float *__restrict__ mean, const float *__restrict__ stdv, float *f) {
    for (int q = threadIdx.x; q < ns * F; q += kNT) {
        int s = q / F, j = q % F;
        int64_t idx = order ? order[s0 + s] : s0 + s;
        float v = feat[idx * F + j];
        if (mean) v = (v - mean[j]) / stdv[j];
        f[s * F + j] = v;
    }
}

__global__ __launch_bounds__(kNT) void k_mlp_forward(const float *__restrict__ gp, const float *__restrict__ feat,
                                                     int64_t m, const float *__restrict__ mean,
                                                     const float *__restrict__ stdv, float *__restrict__ out) {
    __shared__ float p[NP];
    __shared__ float f[kSB * F], z1[kSB * H], z2[kSB * H], o[kSB * K];
    const int64_t s0 = (int64_t)blockIdx.x * kSB;
    const int ns = (int)((m - s0) < kSB ? (m - s0) : kSB);
    load_params(gp, p);
    load_features(feat, nullptr, s0, ns, mean, stdv, f);
    __syncthreads();
    forward_block(p, f, ns, z1, z2, o);
    for (int q = threadIdx.x; q < ns * K; q += kNT) out[s0 * K + q] = o[q];
}

// Per-workgroup partial gradient of L = (1/cnt) sum mask (o - y)^2 over
// samples order[b0 + s0 .. ), and the partial loss sum.  cnt is read from
// *cnt_ptr (mask count of the whole mini-batch).
__global__ __launch_bounds__(kNT) void k_mlp_grad(const float *__restrict__ gp, const float *__restrict__ feat,
                                                  const float *__restrict__ y, const uint8_t *__restrict__ mask,
                                                  const int32_t *__restrict__ order, int64_t b0, int bsz,
                                                  const float *__restrict__ cnt_ptr, float *__restrict__ gpart,
                                                  float *__restrict__ lpart) {
    __shared__ float p[NP];
    __shared__ float f[kSB * F], z1[kSB * H], z2[kSB * H], o[kSB * K];
    __shared__ float go[kSB * K], d2[kSB * H], d1[kSB * H];
    __shared__ float red[kNT];
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * kSB;
    const int ns = (bsz - s0) < kSB ? (bsz - s0) : kSB;
    const float cnt = *cnt_ptr;
    const float inv = cnt > 0.f ? 1.f / cnt : 0.f;
    load_params(gp, p);
    load_features(feat, order, b0 + s0, ns, nullptr, nullptr, f);
    __syncthreads();
    forward_block(p, f, ns, z1, z2, o);
    float lsum = 0.f;
    for (int q = tid; q < ns * K; q += kNT) {
        int s = q / K, k = q % K;
        int64_t idx = order[b0 + s0 + s];
        float e = mask[idx * K + k] ? o[q] - y[idx * K + k] : 0.f;
        lsum += e * e;
        go[q] = 2.f * e * inv;
    }
    red[tid] = lsum;
    __syncthreads();
    for (int d = kNT / 2; d > 0; d >>= 1) {
        if (tid < d) red[tid] += red[tid + d];
        __syncthreads();
    }
    if (tid == 0) lpart[blockIdx.x] = red[0] * inv;
    float *g = gpart + (int64_t)blockIdx.x * NP;
    // layer 3
    for (int q = tid; q < K * H; q += kNT) {
        int k = q / H, j = q % H;
        float a = 0.f;
        for (int s = 0; s < ns; ++s) a += go[s * K + k] * fmaxf(z2[s * H + j], 0.f);
        g[OW3 + q] = a;
    }
    for (int k = tid; k < K; k += kNT) {
        float a = 0.f;
        for (int s = 0; s < ns; ++s) a += go[s * K + k];
        g[OB3 + k] = a;
    }
    for (int q = tid; q < ns * H; q += kNT) {
        int s = q / H, j = q % H;
        float a = 0.f;
        for (int k = 0; k < K; ++k) a += p[OW3 + k * H + j] * go[s * K + k];
        d2[q] = z2[q] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // layer 2
    for (int q = tid; q < H * H; q += kNT) {
        int i = q / H, j = q % H;
        float a = 0.f;
        for (int s = 0; s < ns; ++s) a += d2[s * H + i] * fmaxf(z1[s * H + j], 0.f);
        g[OW2 + q] = a;
    }
    for (int i = tid; i < H; i += kNT) {
        float a = 0.f;
        for (int s = 0; s < ns; ++s) a += d2[s * H + i];
        g[OB2 + i] = a;
    }
    for (int q = tid; q < ns * H; q += kNT) {
        int s = q / H, j = q % H;
        float a = 0.f;
        for (int i = 0; i < H; ++i) a += p[OW2 + i * H + j] * d2[s * H + i];
        d1[q] = z1[q] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // layer 1
    for (int q = tid; q < H * F; q += kNT) {
        int i = q / F, j = q % F;
        float a = 0.f;
        for (int s = 0; s < ns; ++s) a += d1[s * H + i] * f[s * F + j];
        g[OW1 + q] = a;
    }
    for (int i = tid; i < H; i += kNT) {
        float a = 0.f;
        for (int s = 0; s < ns; ++s) a += d1[s * H + i];
        g[OB1 + i] = a;
    }
}

// grad = sum over workgroups (ascending), loss likewise
__global__ void k_mlp_reduce(const float *__restrict__ gpart, const float *__restrict__ lpart, int nb,
                             float *__restrict__ grad, float *__restrict__ loss_out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NP) {
        float a = 0.f;
        for (int b = 0; b < nb; ++b) a += gpart[(int64_t)b * NP + i];
        grad[i] = a;
    }
    if (i == 0 && loss_out) {
        float l = 0.f;
        for (int b = 0; b < nb; ++b) l += lpart[b];
        *loss_out = l;
    }
}

// mask count of the mini-batch order[b0 .. b0 + bsz)
__global__ void k_mask_count(const uint8_t *__restrict__ mask, const int32_t *__restrict__ order, int64_t b0,
                             int bsz, float *__restrict__ cnt) {
    __shared__ int red[kNT];
    int c = 0;
    for (int q = threadIdx.x; q < bsz * K; q += kNT) c += mask[(int64_t)order[b0 + q / K] * K + q % K] ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int d = kNT / 2; d > 0; d >>= 1) {
        if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *cnt = (float)red[0];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// feature mean / std over m samples (one workgroup, fixed order)
__global__ void k_feat_moments(const float *__restrict__ feat, int64_t m, float *__restrict__ mean,
                               float *__restrict__ stdv) {
    __shared__ double s1[kNT], s2[kNT];
    for (int j = 0; j < F; ++j) {
        double a = 0.0, b = 0.0;
        for (int64_t s = threadIdx.x; s < m; s += kNT) {
            double v = feat[s * F + j];
            a += v;
            b += v * v;
        }
        s1[threadIdx.x] = a;
        s2[threadIdx.x] = b;
        __syncthreads();
        for (int d = kNT / 2; d > 0; d >>= 1) {
            if (threadIdx.x < d) {
                s1[threadIdx.x] += s1[threadIdx.x + d];
                s2[threadIdx.x] += s2[threadIdx.x + d];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double mu = s1[0] / (double)m;
            double var = s2[0] / (double)m - mu * mu;
            double sd = var > 0.0 ? sqrt(var) : 0.0;
            mean[j] = (float)mu;
            stdv[j] = sd > 1e-12 ? (float)sd : 1.f;
        }
        __syncthreads();
    }
}

__global__ void k_standardize(const float *__restrict__ feat, int64_t m, const float *__restrict__ mean,
                              const float *__restrict__ stdv, float *__restrict__ out) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m * F) return;
    int j = (int)(q % F);
    out[q] = (feat[q] - mean[j]) / stdv[j];
}

// target y_k = log2(t_k / min over valid t), masked
__global__ void k_targets(const float *__restrict__ cost, const uint8_t *__restrict__ valid, int64_t m,
                          float *__restrict__ y) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    float best = INFINITY;
    for (int k = 0; k < K; ++k)
        if (valid[s * K + k] && cost[s * K + k] < best) best = cost[s * K + k];
    for (int k = 0; k < K; ++k)
        y[s * K + k] = (valid[s * K + k] && best > 0.f) ? log2f(cost[s * K + k] / best) : 0.f;
}

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int upload_model(xab_ctx *ctx) {
    if (!ctx->mlp_set) return xab_fail(ctx, XAB_E_UNSUPPORTED, "no selector model set");
    if (!ctx->d_mlp) {
        ctx->d_mlp = (float *)xab_dalloc(ctx, sizeof(float) * (NP + 2 * F));
        if (!ctx->d_mlp) return xab_fail(ctx, XAB_E_NOMEM, "model");
    }
    XAB_HIP(ctx, hipMemcpyAsync(ctx->d_mlp, ctx->mlp.data(), sizeof(float) * NP, hipMemcpyHostToDevice, ctx->stream));
    XAB_HIP(ctx, hipMemcpyAsync(ctx->d_mlp + NP, ctx->fmean.data(), sizeof(float) * F, hipMemcpyHostToDevice,
                                ctx->stream));
    XAB_HIP(ctx, hipMemcpyAsync(ctx->d_mlp + NP + F, ctx->fstd.data(), sizeof(float) * F, hipMemcpyHostToDevice,
                                ctx->stream));
    return XAB_OK;
}

}  // namespace

// predicted costs of one matrix (used by the LEARNED policy)
int xab_mlp_predict(xab_ctx *ctx, const float *h_feat, float *h_out) {
    int s = upload_model(ctx);
    if (s != XAB_OK) return s;
    float *d = (float *)xab_scratch(ctx, sizeof(float) * (F + K));
    if (!d) return xab_fail(ctx, XAB_E_NOMEM, "scratch");
    XAB_HIP(ctx, hipMemcpyAsync(d, h_feat, sizeof(float) * F, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_mlp_forward, dim3(1), dim3(kNT), 0, ctx->stream, ctx->d_mlp, d, (int64_t)1, ctx->d_mlp + NP,
                       ctx->d_mlp + NP + F, d + F);
    XAB_LAUNCH_CHECK(ctx, "k_mlp_forward");
    XAB_HIP(ctx, hipMemcpyAsync(h_out, d + F, sizeof(float) * K, hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return XAB_OK;
}

extern "C" {

int xab_selector_set(xab_ctx *ctx, const float *h_params, const float *h_mean, const float *h_std) {
    if (!ctx || !h_params || !h_mean || !h_std) return XAB_E_NULL;
    ctx->mlp.assign(h_params, h_params + NP);
    ctx->fmean.assign(h_mean, h_mean + F);
    ctx->fstd.assign(h_std, h_std + F);
    ctx->mlp_set = true;
    return XAB_OK;
}

int xab_selector_get(xab_ctx *ctx, float *h_params, float *h_mean, float *h_std) {
    if (!ctx || !h_params || !h_mean || !h_std) return XAB_E_NULL;
    if (!ctx->mlp_set) return xab_fail(ctx, XAB_E_UNSUPPORTED, "no selector model set");
    memcpy(h_params, ctx->mlp.data(), sizeof(float) * NP);
    memcpy(h_mean, ctx->fmean.data(), sizeof(float) * F);
    memcpy(h_std, ctx->fstd.data(), sizeof(float) * F);
    return XAB_OK;
}

// File format: 8-byte magic "XABSEL01", int32 F, int32 H, int32 K, then
// NP params, F means, F stds as little-endian float32.
int xab_selector_save(xab_ctx *ctx, const char *path) {
    if (!ctx || !path) return XAB_E_NULL;
    if (!ctx->mlp_set) return xab_fail(ctx, XAB_E_UNSUPPORTED, "no selector model set");
    FILE *fp = fopen(path, "wb");
    if (!fp) return xab_fail(ctx, XAB_E_SHAPE, "cannot open %s", path);
    int32_t dims[3] = {F, H, K};
    bool ok = fwrite("XABSEL01", 1, 8, fp) == 8 && fwrite(dims, sizeof(int32_t), 3, fp) == 3 &&
              fwrite(ctx->mlp.data(), sizeof(float), NP, fp) == (size_t)NP &&
              fwrite(ctx->fmean.data(), sizeof(float), F, fp) == (size_t)F &&
              fwrite(ctx->fstd.data(), sizeof(float), F, fp) == (size_t)F;
    fclose(fp);
    return ok ? XAB_OK : xab_fail(ctx, XAB_E_SHAPE, "write failed: %s", path);
}

int xab_selector_load(xab_ctx *ctx, const char *path) {
    if (!ctx || !path) return XAB_E_NULL;
    FILE *fp = fopen(path, "rb");
    if (!fp) return xab_fail(ctx, XAB_E_SHAPE, "cannot open %s", path);
    char magic[8];
    int32_t dims[3];
    std::vector<float> p(NP), mu(F), sd(F);
    bool ok = fread(magic, 1, 8, fp) == 8 && !memcmp(magic, "XABSEL01", 8) && fread(dims, sizeof(int32_t), 3, fp) == 3 &&
              dims[0] == F && dims[1] == H && dims[2] == K && fread(p.data(), sizeof(float), NP, fp) == (size_t)NP &&
              fread(mu.data(), sizeof(float), F, fp) == (size_t)F && fread(sd.data(), sizeof(float), F, fp) == (size_t)F;
    fclose(fp);
    if (!ok) return xab_fail(ctx, XAB_E_SHAPE, "not a selector file: %s", path);
    return xab_selector_set(ctx, p.data(), mu.data(), sd.data());
}

int xab_selector_forward(xab_ctx *ctx, const float *d_feat, int32_t m, int32_t raw, float *d_out) {
    if (!ctx || !d_feat || !d_out) return XAB_E_NULL;
    if (m <= 0) return xab_fail(ctx, XAB_E_SHAPE, "m = %d", m);
    int s = upload_model(ctx);
    if (s != XAB_OK) return s;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(m, kSB)), dim3(kNT), 0, ctx->stream, ctx->d_mlp, d_feat,
                       (int64_t)m, raw ? ctx->d_mlp + NP : nullptr, raw ? ctx->d_mlp + NP + F : nullptr, d_out);
    XAB_LAUNCH_CHECK(ctx, "k_mlp_forward");
    return XAB_OK;
}

int xab_selector_loss_grad(xab_ctx *ctx, const float *d_feat, const float *d_y, const uint8_t *d_valid, int32_t m,
                           float *d_grad, float *loss) {
    if (!ctx || !d_feat || !d_y || !d_valid || !d_grad || !loss) return XAB_E_NULL;
    if (m <= 0) return xab_fail(ctx, XAB_E_SHAPE, "m = %d", m);
    int s = upload_model(ctx);
    if (s != XAB_OK) return s;
    int nb = (int)grid_for(m, kSB);
    size_t need = sizeof(float) * ((size_t)nb * NP + nb + 2) + sizeof(int32_t) * (size_t)m;
    char *w = (char *)xab_scratch(ctx, need);
    if (!w) return xab_fail(ctx, XAB_E_NOMEM, "scratch");
    float *gpart = (float *)w, *lpart = gpart + (size_t)nb * NP, *cnt = lpart + nb, *lout = cnt + 1;
    int32_t *order = (int32_t *)(lout + 1);
    std::vector<int32_t> h(m);
    for (int i = 0; i < m; ++i) h[i] = i;
    XAB_HIP(ctx, hipMemcpyAsync(order, h.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_mask_count, dim3(1), dim3(kNT), 0, ctx->stream, d_valid, order, (int64_t)0, m, cnt);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kNT), 0, ctx->stream, ctx->d_mlp, d_feat, d_y, d_valid, order,
                       (int64_t)0, m, cnt, gpart, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(NP, 256)), dim3(256), 0, ctx->stream, gpart, lpart, nb, d_grad, lout);
    XAB_LAUNCH_CHECK(ctx, "mlp gradient");
    XAB_HIP(ctx, hipMemcpyAsync(loss, lout, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return XAB_OK;
}

int xab_selector_train(xab_ctx *ctx, const float *d_feat, const float *d_cost, const uint8_t *d_valid, int32_t m,
                       const int32_t *h_order, const xab_train_opts *opts, float *h_loss, xab_train_info *info) {
    if (!ctx || !d_feat || !d_cost || !d_valid || !h_order || !opts) return XAB_E_NULL;
    if (m <= 0 || opts->epochs <= 0 || opts->batch <= 0) return xab_fail(ctx, XAB_E_SHAPE, "bad training sizes");
    if (!ctx->mlp_set) return xab_fail(ctx, XAB_E_UNSUPPORTED, "set initial parameters first");
    auto t0 = std::chrono::steady_clock::now();
    const int E = opts->epochs, B = opts->batch;
    const int nbat = (m + B - 1) / B;
    const int nbw = (int)grid_for(B, kSB);
    // workspace
    size_t fl = (size_t)m * F + (size_t)m * K + 3 * (size_t)NP + 2 * F + (size_t)nbw * NP + nbw + 1 +
                (size_t)E * nbat;
    float *w = (float *)xab_dalloc(ctx, sizeof(float) * fl);
    int32_t *d_order = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)E * m);
    if (!w || !d_order) {
        xab_dfree(ctx, w);
        xab_dfree(ctx, d_order);
        return xab_fail(ctx, XAB_E_NOMEM, "training workspace");
    }
    float *fs = w, *y = fs + (size_t)m * F, *p = y + (size_t)m * K, *mo = p + NP, *ve = mo + NP;
    float *mean = ve + NP, *stdv = mean + F, *gpart = stdv + F, *lpart = gpart + (size_t)nbw * NP;
    float *cnt = lpart + nbw, *losses = cnt + 1;
    float *grad = (float *)xab_scratch(ctx, sizeof(float) * NP);
    int st = XAB_OK;
    auto fail = [&](int code) {
        xab_dfree(ctx, w);
        xab_dfree(ctx, d_order);
        return code;
    };
    if (!grad) return fail(xab_fail(ctx, XAB_E_NOMEM, "scratch"));
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(d_order, h_order, sizeof(int32_t) * (size_t)E * m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(p, ctx->mlp.data(), sizeof(float) * NP, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(mo, 0, sizeof(float) * 2 * NP, s);
    if (e != hipSuccess) return fail(xab_hip_check(ctx, e, "training setup"));
    hipLaunchKernelGGL(k_feat_moments, dim3(1), dim3(kNT), 0, s, d_feat, (int64_t)m, mean, stdv);
    hipLaunchKernelGGL(k_standardize, dim3(grid_for((int64_t)m * F, 256)), dim3(256), 0, s, d_feat, (int64_t)m, mean,
                       stdv, fs);
    hipLaunchKernelGGL(k_targets, dim3(grid_for(m, 256)), dim3(256), 0, s, d_cost, d_valid, (int64_t)m, y);
    int64_t t = 0;
    for (int ep = 0; ep < E; ++ep) {
        for (int bi = 0; bi < nbat; ++bi) {
            int64_t b0 = (int64_t)ep * m + (int64_t)bi * B;
            int bsz = (m - bi * B) < B ? (m - bi * B) : B;
            int nb = (int)grid_for(bsz, kSB);
            hipLaunchKernelGGL(k_mask_count, dim3(1), dim3(kNT), 0, s, d_valid, d_order, b0, bsz, cnt);
            hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kNT), 0, s, p, fs, y, d_valid, d_order, b0, bsz, cnt, gpart,
                               lpart);
            hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(NP, 256)), dim3(256), 0, s, gpart, lpart, nb, grad,
                               losses + (int64_t)ep * nbat + bi);
            ++t;
            float c1 = (float)(1.0 - std::pow((double)opts->beta1, (double)t));
            float c2 = (float)(1.0 - std::pow((double)opts->beta2, (double)t));
            hipLaunchKernelGGL(k_adam, dim3(grid_for(NP, 256)), dim3(256), 0, s, p, grad, mo, ve, opts->lr, opts->beta1,
                               opts->beta2, opts->eps, c1, c2);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return fail(xab_hip_check(ctx, e, "training step"));
    }
    std::vector<float> hl((size_t)E * nbat);
    std::vector<float> hm(F), hs(F);
    e = hipMemcpyAsync(ctx->mlp.data(), p, sizeof(float) * NP, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hl.data(), losses, sizeof(float) * hl.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hm.data(), mean, sizeof(float) * F, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), stdv, sizeof(float) * F, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(xab_hip_check(ctx, e, "training read-back"));
    ctx->fmean = hm;
    ctx->fstd = hs;
    float last = 0.f;
    for (int ep = 0; ep < E; ++ep) {
        double a = 0.0;
        for (int bi = 0; bi < nbat; ++bi) a += hl[(size_t)ep * nbat + bi];
        float le = (float)(a / nbat);
        if (h_loss) h_loss[ep] = le;
        last = le;
    }
    if (info) {
        info->final_loss = last;
        info->seconds = (float)std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    (void)st;
    return fail(XAB_OK);
}

}  // extern "C"
