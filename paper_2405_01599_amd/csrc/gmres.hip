// Restarted GMRES(m) with right Jacobi preconditioning, in FP64 or as
// mixed-precision iterative refinement (FP32 values and basis inside, FP64
// residuals, inner products and Hessenberg/Givens outside).
//
// Orthogonalisation: classical Gram-Schmidt with the DGKS re-orthogonali-
// sation test (a second CGS pass when ||w'|| < ||w|| / sqrt(2)), one of the
// four orthogonalisers of the paper's section 3.2.2.  Each pass is one fused
// multi-dot over all basis vectors plus one fused update, so a step costs
// two or four sweeps of the basis instead of the 2j of modified GS.
//
// Convergence is declared only on the true residual ||b - A x|| / ||b||,
// computed in FP64 at every restart: the recurrence estimate only ends a
// cycle (the accuracy policy's outer check against "fault convergence",
// section 3.3.2).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "blas.h"

namespace {

constexpr double kEta = 0.70710678118654752440;  // DGKS threshold 1/sqrt(2)

struct Work {
    xab_ctx *ctx = nullptr;
    void *base = nullptr;
    double *r = nullptr;     // FP64 residual / product buffer [n]
    double *part = nullptr;  // partial sums [kRedBlocks * kPartLd]
    double *h1 = nullptr, *h2 = nullptr, *sc = nullptr;  // small device vectors
    int *gate = nullptr;
    void *V = nullptr, *w = nullptr, *z = nullptr;
    int64_t ldv = 0;
    size_t small_bytes = 0;  // h1 .. gate, read back in one copy per step
    double *host = nullptr;  // pinned mirror of that region
    ~Work() {
        if (base) xab_dfree(ctx, base);
        if (host) (void)hipHostFree(host);
    }
};

int alloc_work(xab_ctx *ctx, Work &W, int64_t n, int m, size_t tsize) {
    W.ctx = ctx;
    W.ldv = (n + 63) / 64 * 64;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off_r = 0, off_part = off_r + al(sizeof(double) * n);
    size_t off_small = off_part + al(sizeof(double) * xab::kRedBlocks * xab::kPartLd);
    size_t off_V = off_small + al(sizeof(double) * (3 * (m + 2) + 16) + 64);
    size_t off_w = off_V + al(tsize * (size_t)(m + 1) * W.ldv);
    size_t off_z = off_w + al(tsize * W.ldv);
    size_t total = off_z + al(tsize * W.ldv);
    char *b = (char *)xab_dalloc(ctx, total);
    if (!b) return xab_fail(ctx, XAB_E_NOMEM, "GMRES workspace (%zu bytes)", total);
    W.base = b;
    W.r = (double *)(b + off_r);
    W.part = (double *)(b + off_part);
    W.h1 = (double *)(b + off_small);
    W.h2 = W.h1 + (m + 2);
    W.sc = W.h2 + (m + 2);
    W.gate = (int *)(W.sc + (m + 2) + 8);
    W.V = b + off_V;
    W.w = b + off_w;
    W.z = b + off_z;
    W.small_bytes = sizeof(double) * (3 * (size_t)(m + 2) + 8) + sizeof(int);
    if (hipHostMalloc((void **)&W.host, W.small_bytes, hipHostMallocDefault) != hipSuccess) {
        W.host = nullptr;
        return xab_fail(ctx, XAB_E_NOMEM, "pinned host buffer");
    }
    return XAB_OK;
}

struct Cycle {
    int k = 0;               // Arnoldi steps taken
    double est = 0.0;        // recurrence residual estimate |g_{k}|
    bool breakdown = false;  // h_{j+1,j} = 0
    std::vector<double> samp;  // |g_0| = beta, then |g_{j+1}| after every step
    bool by_recurrence = false;  // ended because the recurrence residual met the threshold
};

// The MM ratio of eq. (1) over samples v[s-t .. s-1]: max / min.
double mm_ratio(const std::vector<double> &v, size_t s, size_t t) {
    double mx = v[s - t], mn = v[s - t];
    for (size_t z = s - t; z < s; ++z) {
        mx = std::max(mx, v[z]);
        mn = std::min(mn, v[z]);
    }
    return mx / mn;
}

// One GMRES(m) cycle on A M^-1 u = rhs where rhs = r (FP64, ||r|| = beta),
// basis in T.  Stops after m steps, at a lucky breakdown or when the
// recurrence residual falls to tol_abs.  Adds scale * M^-1 V y to x.
template <class T>
int cycle(xab_ctx *ctx, const xab_plan *pl, xab_matrix *A, Work &W, int m, double beta, double tol_abs,
          int64_t max_steps, double *x, int ortho, Cycle &out) {
    const int64_t n = A->n;
    const T *d = nullptr;
    if constexpr (sizeof(T) == 8) d = (const T *)A->diag64;
    else d = (const T *)A->diag32;
    T *V = (T *)W.V, *w = (T *)W.w, *z = (T *)W.z;
    const xab_dtype tt = sizeof(T) == 8 ? XAB_F64 : XAB_F32;
    const int nb = xab::kRedBlocks;
    int s;
    // v0 = r / beta, z = M^-1 v0
    if ((s = xab::scale_from<double, T>(ctx, W.r, 1.0 / beta, V, z, d, n)) != XAB_OK) return s;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0);
    g[0] = beta;
    out.samp.assign(1, beta);
    int k = 0;
    out.breakdown = false;
    for (int j = 0; j < m && j < max_steps; ++j) {
        // w = A z (FP64 accumulation in every mode)
        if ((s = xab_spmv_dispatch(ctx, pl, z, tt, w, tt, XAB_F64)) != XAB_OK) return s;
        const size_t oh2 = (size_t)(W.h2 - W.h1), osc = (size_t)(W.sc - W.h1);  // layout of the small region
        bool dgks = false;
        if (ortho == XAB_ORTHO_DGKS) {
            // pass 1: h1 = V^T w, ||w||^2; then one sweep: w' = w - V h1 with
            // the second pass's h2 = V^T w', ||w'||^2 from the same reads of V
            dgks = true;
            if ((s = xab::mdot<T>(ctx, V, W.ldv, j + 1, w, n, W.part, nb, nullptr)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, j + 2, W.h1, 0, nullptr)) != XAB_OK) return s;
            if ((s = xab::update_mdot<T>(ctx, V, j + 1, W.h1, V, j + 1, W.ldv, w, n, W.part, nb)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, j + 2, W.h2, 0, nullptr)) != XAB_OK) return s;
            // the second update only when cancellation was severe
            if ((s = xab::dgks_gate(ctx, W.h1 + j + 1, W.h2 + j + 1, kEta, W.gate)) != XAB_OK) return s;
            if ((s = xab::update_norm<T>(ctx, V, W.ldv, j + 1, W.h2, w, n, W.part, nb, W.gate)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, 1, 1, W.sc, 0, W.gate)) != XAB_OK) return s;
        } else if (ortho == XAB_ORTHO_CGS) {
            // h1 = V^T w, then w -= V h1; ||w||^2 into h1[j+1]
            if ((s = xab::mdot<T>(ctx, V, W.ldv, j + 1, w, n, W.part, nb, nullptr)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, j + 1, W.h1, 0, nullptr)) != XAB_OK) return s;
            if ((s = xab::update_norm<T>(ctx, V, W.ldv, j + 1, W.h1, w, n, W.part, nb, nullptr)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, 1, 1, W.h1 + j + 1, 0, nullptr)) != XAB_OK) return s;
        } else {
            // MGS (blocks of one column) or BCGS (blocks of four): each
            // sweep applies one block's update and forms the next block's
            // dots with the updated w; the last sweep leaves ||w||^2 in h1[j+1]
            const int bs = ortho == XAB_ORTHO_MGS ? 1 : 4;
            const int nb0 = std::min(bs, j + 1);
            if ((s = xab::mdot<T>(ctx, V, W.ldv, nb0, w, n, W.part, nb, nullptr)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, nb0, W.h1, 0, nullptr)) != XAB_OK) return s;
            for (int b0 = 0; b0 <= j; b0 += bs) {
                const int b1 = std::min(b0 + bs, j + 1);
                const int c1 = std::min(b1 + bs, j + 1);  // next block [b1, c1)
                const T *Vn = c1 > b1 ? V + (int64_t)b1 * W.ldv : nullptr;
                if ((s = xab::update_mdot<T>(ctx, V + (int64_t)b0 * W.ldv, b1 - b0, W.h1 + b0, Vn, c1 - b1, W.ldv, w,
                                             n, W.part, nb)) != XAB_OK)
                    return s;
                if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, c1 - b1 + 1, W.h1 + b1, 0, nullptr)) !=
                    XAB_OK)
                    return s;
            }
        }
        // v_{j+1} = w / ||w||, z = M^-1 v_{j+1}
        T *vn = V + (int64_t)(j + 1) * W.ldv;
        if (dgks) {
            if ((s = xab::scale_precond<T>(ctx, w, W.h2 + j + 1, vn, z, d, n, W.sc, W.gate)) != XAB_OK) return s;
        } else {
            if ((s = xab::scale_precond<T>(ctx, w, W.h1 + j + 1, vn, z, d, n)) != XAB_OK) return s;
        }
        // one read-back of the coefficients, the norms and the DGKS gate (contiguous)
        XAB_HIP(ctx, hipMemcpyAsync(W.host, W.h1, W.small_bytes, hipMemcpyDeviceToHost, ctx->stream));
        XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const double *hh = W.host;
        int gate = 0;
        if (dgks) memcpy(&gate, (const char *)W.gate - (const char *)W.h1 + (const char *)W.host, sizeof(int));
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + (gate ? hh[oh2 + i] : 0.0);
        const double hn = std::sqrt(!dgks ? hh[j + 1] : (gate ? hh[osc] : hh[oh2 + j + 1]));
        H[(size_t)(j + 1) * m + j] = hn;
        // earlier rotations on column j, then a new one
        for (int i = 0; i < j; ++i) {
            double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
            H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
        }
        double a = H[(size_t)j * m + j], c = hn;
        double rr = std::hypot(a, c);
        cs[j] = rr == 0.0 ? 1.0 : a / rr;
        sn[j] = rr == 0.0 ? 0.0 : c / rr;
        H[(size_t)j * m + j] = rr;
        H[(size_t)(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        k = j + 1;
        out.samp.push_back(std::fabs(g[j + 1]));
        if (hn == 0.0) {
            out.breakdown = true;
            break;
        }
        if (std::fabs(g[j + 1]) <= tol_abs) {
            out.by_recurrence = true;
            break;
        }
    }
    // back substitution on the rotated triangle
    std::vector<double> y(k > 0 ? k : 1, 0.0);
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q < k; ++q) t -= H[(size_t)i * m + q] * y[q];
        y[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
    }
    out.k = k;
    out.est = std::fabs(g[k]);
    if (k > 0) {
        XAB_HIP(ctx, hipMemcpyAsync(W.h2, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
        if ((s = xab::combine<T>(ctx, V, W.ldv, k, W.h2, 1.0, d, x, n)) != XAB_OK) return s;
    }
    return XAB_OK;
}

// r = b - A x in FP64; returns ||r||
int true_residual(xab_ctx *ctx, const xab_plan *pl, const double *b, const double *x, Work &W, int64_t n,
                  double *nrm) {
    int s = xab_spmv_dispatch(ctx, pl, x, XAB_F64, W.r, XAB_F64, XAB_F64);
    if (s != XAB_OK) return s;
    if ((s = xab::residual(ctx, b, W.r, n, W.part, xab::kRedBlocks)) != XAB_OK) return s;
    if ((s = xab::reduce_parts(ctx, W.part, xab::kRedBlocks, 1, 1, W.sc, 0, nullptr)) != XAB_OK) return s;
    double h = 0.0;
    XAB_HIP(ctx, hipMemcpyAsync(&h, W.sc, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *nrm = std::sqrt(h);
    return XAB_OK;
}

}  // namespace

extern "C" int xab_gmres(xab_ctx *ctx, const xab_plan *pl, const double *d_b, double *d_x, const xab_krylov_opts *opts,
                         xab_krylov_info *info) {
    if (!ctx || !pl || !d_b || !d_x || !opts) return XAB_E_NULL;
    xab_matrix *A = const_cast<xab_matrix *>(pl->A);  // caches the Jacobi diagonal
    if (A->n != A->ncols) return xab_fail(ctx, XAB_E_SHAPE, "GMRES needs a square matrix");
    const int m0 = opts->m;
    if (m0 < 1 || m0 > 63) return xab_fail(ctx, XAB_E_SHAPE, "restart length must be in [1, 63]");
    const bool tune = opts->restart_step > 0 && ctx->policy != XAB_MEMORY;  // MEMORY: the basis keeps its size
    if (tune && (opts->m_max < m0 || opts->m_max > 63))
        return xab_fail(ctx, XAB_E_SHAPE, "m_max must be in [m, 63]");
    const int mcap = tune ? opts->m_max : m0;  // basis capacity
    int m = m0;                                // restart length of the next cycle
    if (opts->ortho < XAB_ORTHO_DGKS || opts->ortho > XAB_ORTHO_POLICY) return xab_fail(ctx, XAB_E_SHAPE, "ortho");
    // on an ACCURACY context the accuracy policy's rule replaces the choice
    const bool policy = opts->ortho == XAB_ORTHO_POLICY || ctx->policy == XAB_ACCURACY;
    // the policy's rule applies to the requirement of the solve being
    // orthogonalised: the FP64 solve's tol, or in IR mode the inner tolerance
    const double req = opts->mode == XAB_MODE_IR ? (opts->inner_tol > 0 ? opts->inner_tol : 1e-6) : opts->tol;
    int ortho = policy ? (req <= 1e-10 ? XAB_ORTHO_MGS : XAB_ORTHO_BCGS) : opts->ortho;
    double rec_scale = 1.0;  // the policy narrows the recurrence threshold after a fault
    bool last_by_rec = false;
    if (opts->mode != XAB_MODE_FP64 && opts->mode != XAB_MODE_IR) return xab_fail(ctx, XAB_E_SHAPE, "mode");
    if (!A->has64) return xab_fail(ctx, XAB_E_DTYPE, "GMRES needs FP64 values for the residual");
    if (opts->mode == XAB_MODE_IR && !A->has32) return xab_fail(ctx, XAB_E_DTYPE, "IR mode needs FP32 values");
    if (opts->mode == XAB_MODE_IR && pl->variant == XAB_SYM_ATOMIC)
        return xab_fail(ctx, XAB_E_DTYPE, "IR mode's inner product (FP32 y, FP64 accumulation) has no atomic form");
    if (d_b == d_x) return xab_fail(ctx, XAB_E_ALIAS, "b and x alias");
    const int64_t n = A->n;
    xab_krylov_info loc{};
    xab_krylov_info &inf = info ? *info : loc;
    inf = xab_krylov_info{};
    if (n == 0) return XAB_OK;
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    int s;
    if (opts->precond == XAB_PRECOND_JACOBI && (s = xab_matrix_diag(ctx, A)) != XAB_OK) return s;
    const bool jac = opts->precond == XAB_PRECOND_JACOBI;
    // the cycle reads the diagonal from A; hide it when not preconditioning
    double *d64 = A->diag64;
    float *d32 = A->diag32;
    if (!jac) {
        A->diag64 = nullptr;
        A->diag32 = nullptr;
    }
    struct Restore {
        xab_matrix *A;
        double *d64;
        float *d32;
        ~Restore() {
            A->diag64 = d64;
            A->diag32 = d32;
        }
    } restore{A, d64, d32};
    Work W;
    const bool ir = opts->mode == XAB_MODE_IR;
    if ((s = alloc_work(ctx, W, n, mcap, ir ? sizeof(float) : sizeof(double))) != XAB_OK) return s;
    auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    // ||b||
    if ((s = xab::mdot<double>(ctx, nullptr, 0, 0, d_b, n, W.part, xab::kRedBlocks, nullptr)) != XAB_OK) return s;
    if ((s = xab::reduce_parts(ctx, W.part, xab::kRedBlocks, xab::kPartLd, 1, W.sc, 0, nullptr)) != XAB_OK) return s;
    double bn2 = 0.0;
    XAB_HIP(ctx, hipMemcpyAsync(&bn2, W.sc, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double bn = std::sqrt(bn2);
    if (bn == 0.0) bn = 1.0;
    const int64_t maxiter = opts->maxiter > 0 ? opts->maxiter : INT64_MAX;
    int status = XAB_NOT_CONVERGED;
    double relres = 0.0;
    for (;;) {
        double beta = 0.0;
        if ((s = true_residual(ctx, pl, d_b, d_x, W, n, &beta)) != XAB_OK) return s;
        relres = beta / bn;
        if (relres <= opts->tol) {
            status = XAB_OK;
            break;
        }
        if (last_by_rec && policy && !ir) {
            // fault convergence: the recurrence met the threshold, the true residual did not
            inf.faults++;
            ortho = XAB_ORTHO_DGKS;
            rec_scale *= 0.1;
        }
        last_by_rec = false;
        if (inf.iters >= maxiter) break;
        if (opts->max_time_s > 0 && elapsed() > opts->max_time_s) {
            status = XAB_TIME_LIMIT;
            break;
        }
        Cycle c;
        if (ir) {
            // inner solve of A d = r to inner_tol (or one cycle), then x += d
            double inner = opts->inner_tol > 0 ? opts->inner_tol : 1e-6;
            double tol_abs = std::max(inner * beta, 0.1 * opts->tol * bn);
            s = cycle<float>(ctx, pl, A, W, m, beta, tol_abs, maxiter - inf.iters, d_x, ortho, c);
            inf.refinements++;
        } else {
            s = cycle<double>(ctx, pl, A, W, m, beta, opts->tol * bn * rec_scale, maxiter - inf.iters, d_x, ortho, c);
        }
        last_by_rec = c.by_recurrence;
        if (s != XAB_OK) return s;
        inf.iters += c.k;
        inf.restarts++;
        inf.m_final = m;
        if (c.k == 0) break;
        // restart-length judgment on this cycle's residual samples (relative
        // to ||b||; the ratio is scale-free)
        if (tune && m < opts->m_max && mm_ratio(c.samp, c.samp.size(), c.samp.size()) < opts->mm_ratio)
            m = std::min(m + opts->restart_step, opts->m_max);
    }
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    inf.true_relres = relres;
    inf.seconds = elapsed();
    inf.status = status;
    inf.ortho = ortho;
    return status;
}
