// The run-time judge: choose one SpMV implementation for a matrix.
//   TIME     every valid class is set up and measured (1 warm-up, 4 timed
//            runs, minimum kept); the fastest wins, ties to the lowest class
//            (the before-execution auto-tuning of the paper's section 3.1)
//   STABLE   no tuning: a fixed default (section 2.3, policy STABLE)
//   LEARNED  the cost model predicts every class from the matrix features;
//            the best predicted class that can be set up wins
//   ACCURACY as TIME (the implementation changes the product only by
//            rounding; the policy acts in the solvers)
//   MEMORY   the least device memory (section 2.3, policy MEMORY): every
//            valid class is set up once to learn its plan's bytes; those
//            within 1/64 of the matrix's own bytes of the least are timed as
//            under TIME and the fastest of them wins
#include <chrono>
#include <cmath>

#include "internal.h"

int xab_mlp_predict(xab_ctx *ctx, const float *h_feat, float *h_out);

namespace {

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float *p, int64_t n, float v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

bool class_applies(int k, bool sym) { return sym ? (k >= 9 && k <= 11) : (k < 9 || k >= 12); }

// class k with time t displaces the best so far (kb, tb): faster, or as
// fast with a lower index
bool displaces(float t, int k, float tb, int kb) { return kb < 0 || t < tb || (t == tb && k < kb); }

constexpr int kStableGeneral = 3, kStableSym = 11, kStableSymFallback = 9;

}  // namespace

extern "C" int xab_select(xab_ctx *ctx, const xab_matrix *A, xab_policy policy, xab_plan **out, xab_select_info *info) {
    if (!ctx || !A || !out) return XAB_E_NULL;
    *out = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    xab_select_info loc{};
    xab_select_info &inf = info ? *info : loc;
    inf = xab_select_info{};
    for (int k = 0; k < XAB_NCLASSES; ++k) {
        inf.time_ms[k] = -1.f;
        inf.valid[k] = class_applies(k, A->sym()) ? 1 : 0;
        inf.bytes[k] = -1;
    }
    inf.chosen = -1;
    const bool sym = A->sym();
    auto finish = [&](xab_plan *pl, int k) {
        *out = pl;
        inf.chosen = k;
        inf.select_ms = (float)(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        return XAB_OK;
    };
    auto build = [&](int k, xab_plan **pl) {
        xab_variant v;
        xab_params p;
        xab_class_params(k, &v, &p);
        return xab_build_plan(ctx, A, v, &p, pl);
    };

    if (policy == XAB_STABLE) {
        int k = sym ? kStableSym : kStableGeneral;
        xab_plan *pl = nullptr;
        int s = build(k, &pl);
        if (s == XAB_E_UNSUPPORTED && sym) {
            inf.valid[k] = 0;
            k = kStableSymFallback;
            s = build(k, &pl);
        }
        if (s != XAB_OK) return s;
        return finish(pl, k);
    }

    if (policy == XAB_LEARNED) {
        if (A->n == 0) return xab_fail(ctx, XAB_E_SHAPE, "empty matrix");
        float feat[12], pred[XAB_NCLASSES];
        int s = xab_features(ctx, A, feat, nullptr);
        if (s != XAB_OK) return s;
        s = xab_mlp_predict(ctx, feat, pred);
        if (s != XAB_OK) return s;
        for (int k = 0; k < XAB_NCLASSES; ++k)
            if (inf.valid[k]) inf.time_ms[k] = pred[k];
        // best predicted class that can be set up (lowest index on ties)
        for (int tries = 0; tries < XAB_NCLASSES; ++tries) {
            int best = -1;
            for (int k = 0; k < XAB_NCLASSES; ++k)
                if (inf.valid[k] && (best < 0 || pred[k] < pred[best])) best = k;
            if (best < 0) break;
            xab_plan *pl = nullptr;
            s = build(best, &pl);
            if (s == XAB_OK) return finish(pl, best);
            if (s != XAB_E_UNSUPPORTED) return s;
            inf.valid[best] = 0;
            inf.time_ms[best] = -1.f;
        }
        return xab_fail(ctx, XAB_E_UNSUPPORTED, "no applicable SpMV class");
    }

    // ACCURACY: the SpMV implementation does not change what is computed
    // beyond rounding, so it is chosen as under TIME
    if (policy == XAB_ACCURACY) policy = XAB_TIME;
    if (policy != XAB_TIME && policy != XAB_MEMORY) return xab_fail(ctx, XAB_E_SHAPE, "unknown policy %d", (int)policy);
    // MEMORY: the plan bytes of every valid class first; only the classes
    // within the slack of the least are timed below
    bool timed[XAB_NCLASSES];
    for (int k = 0; k < XAB_NCLASSES; ++k) timed[k] = inf.valid[k] != 0;
    if (policy == XAB_MEMORY) {
        int64_t least = -1;
        for (int k = 0; k < XAB_NCLASSES; ++k) {
            if (!inf.valid[k]) continue;
            xab_plan *pl = nullptr;
            int s = build(k, &pl);
            if (s == XAB_E_UNSUPPORTED) {
                inf.valid[k] = 0;
                timed[k] = false;
                continue;
            }
            if (s != XAB_OK) return s;
            inf.bytes[k] = xab_plan_bytes(pl);
            xab_plan_destroy(pl);
            if (least < 0 || inf.bytes[k] < least) least = inf.bytes[k];
        }
        const int64_t own = 4 * ((int64_t)A->n + 1) + A->nnz * (4 + (A->has64 ? 8 : 4));
        for (int k = 0; k < XAB_NCLASSES; ++k) timed[k] = inf.valid[k] && inf.bytes[k] <= least + own / 64;
    }
    // TIME: measure every valid class (MEMORY: the classes kept above)
    const bool f64 = A->has64;
    const size_t es = f64 ? 8 : 4;
    const int64_t nx = A->ncols, ny = A->n;
    char *buf = (char *)xab_dalloc(ctx, es * (size_t)(nx + ny) + 256);
    if (!buf) return xab_fail(ctx, XAB_E_NOMEM, "selector vectors");
    void *x = buf;
    void *y = buf + ((es * nx + 255) / 256) * 256;
    if (f64) hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((nx + 255) / 256 + 1)), dim3(256), 0, ctx->stream, (double *)x, nx, 1.0);
    else hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((nx + 255) / 256 + 1)), dim3(256), 0, ctx->stream, (float *)x, nx, 1.f);
    xab_dtype dt = f64 ? XAB_F64 : XAB_F32;
    hipEvent_t ev[5];
    for (auto &e : ev) (void)hipEventCreate(&e);
    xab_plan *best_plan = nullptr;
    int best = -1, status = XAB_OK;
    for (int k = 0; k < XAB_NCLASSES && status == XAB_OK; ++k) {
        if (!timed[k]) continue;
        xab_plan *pl = nullptr;
        int s = build(k, &pl);
        if (s == XAB_E_UNSUPPORTED) {
            inf.valid[k] = 0;
            continue;
        }
        if (s != XAB_OK) {
            status = s;
            break;
        }
        inf.bytes[k] = xab_plan_bytes(pl);
        s = xab_spmv_dispatch(ctx, pl, x, dt, y, dt, dt);  // warm-up
        float tmin = INFINITY;
        for (int r = 0; r < 4 && s == XAB_OK; ++r) {
            (void)hipEventRecord(ev[r], ctx->stream);
            s = xab_spmv_dispatch(ctx, pl, x, dt, y, dt, dt);
            (void)hipEventRecord(ev[r + 1], ctx->stream);
            hipError_t e = hipEventSynchronize(ev[r + 1]);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
            if (e != hipSuccess) s = xab_hip_check(ctx, e, "selector timing");
            tmin = ms < tmin ? ms : tmin;
        }
        if (s != XAB_OK) {
            xab_plan_destroy(pl);
            status = s;
            break;
        }
        inf.time_ms[k] = tmin;
        if (displaces(tmin, k, best < 0 ? 0.f : inf.time_ms[best], best)) {
            if (best_plan) xab_plan_destroy(best_plan);
            best_plan = pl;
            best = k;
        } else {
            xab_plan_destroy(pl);
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    (void)hipStreamSynchronize(ctx->stream);
    xab_dfree(ctx, buf);
    if (status != XAB_OK) {
        if (best_plan) xab_plan_destroy(best_plan);
        return status;
    }
    if (!best_plan) return xab_fail(ctx, XAB_E_UNSUPPORTED, "no applicable SpMV class");
    return finish(best_plan, best);
}

extern "C" int xab_select_rule(const float *time_ms, const int32_t *valid, int32_t n, int32_t *chosen) {
    if (!chosen) return XAB_E_NULL;
    *chosen = -1;
    if (n < 0) return XAB_E_SHAPE;
    if (n > 0 && (!time_ms || !valid)) return XAB_E_NULL;
    int best = -1;
    for (int k = 0; k < n; ++k) {
        const float t = time_ms[k];
        if (!valid[k] || !(t >= 0.f) || std::isinf(t)) continue;
        if (displaces(t, k, best < 0 ? 0.f : time_ms[best], best)) best = k;
    }
    *chosen = best;
    return best < 0 ? XAB_E_UNSUPPORTED : XAB_OK;
}

extern "C" int xab_class_applies(int32_t k, int32_t sym) {
    if (k < 0 || k >= XAB_NCLASSES) return XAB_E_SHAPE;
    return class_applies(k, sym != 0) ? 1 : 0;
}
