// Restarted Lanczos for the symmetric standard eigenproblem (the solver
// list of section 2.2; the setting of section 4.3: 10 eigenpairs, accuracy
// 1e-8).  The restart scheme is the thick restart of Wu and Simon (2000):
// after m basis vectors the Ritz pairs of T = Q^T A Q are formed, the k
// wanted ones nearest the chosen end are kept as the first k basis vectors
// and the recurrence continues from the residual direction.
//
// Device side: the products with A go through the plan (any variant,
// general or lower-stored), every new vector is orthogonalised against the
// whole basis by classical Gram-Schmidt with the DGKS second pass, and the
// coefficients of every step are left in device slots, so a cycle of m
// steps runs without a host round trip.  Host side, once per cycle: T
// (arrowhead + tridiagonal, at most 63 x 63) is diagonalised by cyclic
// Jacobi and the restart or the final eigenvectors are formed by one
// basis rotation kernel.
#include "eig_common.h"

namespace {

// Cyclic Jacobi for a symmetric n x n matrix (row-major a, destroyed):
// rotations J(p, q, theta) zeroing a_pq in row order until the off-diagonal
// Frobenius norm is below 1e-17 of the whole (Golub and Van Loan, the
// cyclic Jacobi algorithm).  w receives the eigenvalues, z (row-major) the
// eigenvectors as columns.
void jacobi_eig(int n, std::vector<double> &a, std::vector<double> &w, std::vector<double> &z) {
    z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    auto A = [&](int i, int j) -> double & { return a[(size_t)i * n + j]; };
    double fro = 0.0;
    for (double v : a) fro += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) off += A(i, j) * A(i, j);
        if (off <= 1e-34 * fro || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                // symmetric 2 x 2 Schur decomposition: t = tan(theta), the smaller root
                const double tau = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                A(p, q) = A(q, p) = 0.0;
                for (int k = 0; k < n; ++k) {  // Z <- Z J
                    const double zkp = z[(size_t)k * n + p], zkq = z[(size_t)k * n + q];
                    z[(size_t)k * n + p] = c * zkp - s * zkq;
                    z[(size_t)k * n + q] = s * zkp + c * zkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A(i, i);
}

}  // namespace

extern "C" int xab_lanczos(xab_ctx *ctx, const xab_plan *pl, const double *d_v0, const xab_eig_opts *opts,
                           double *h_evals, double *d_evecs, xab_eig_info *info) {
    if (!ctx || !pl || !d_v0 || !opts) return XAB_E_NULL;
    const xab_matrix *A = pl->A;
    const int64_t n = A->n;
    const int nev = opts->nev;
    int m = opts->m;  // length of the next cycle
    const bool tune = opts->restart_step > 0 && ctx->policy != XAB_MEMORY;  // MEMORY: the basis keeps its size
    const int mc = tune ? opts->m_max : m;  // basis capacity
    const int window = opts->window > 0 ? opts->window : 5;
    if (A->n != A->ncols) return xab_fail(ctx, XAB_E_SHAPE, "Lanczos needs a square matrix");
    if (nev < 1 || m <= nev || m > kMaxM || m > n)
        return xab_fail(ctx, XAB_E_SHAPE, "need 1 <= nev < m <= min(63, n) (nev %d, m %d, n %lld)", nev, m,
                        (long long)n);
    if (tune && (mc < m || mc > kMaxM || mc > n))
        return xab_fail(ctx, XAB_E_SHAPE, "m_max must be in [m, min(63, n)] (m_max %d)", mc);
    if (opts->which != XAB_EIG_LARGEST && opts->which != XAB_EIG_SMALLEST)
        return xab_fail(ctx, XAB_E_SHAPE, "which");
    if (!h_evals || !d_evecs) return XAB_E_NULL;
    if (!A->has64) return xab_fail(ctx, XAB_E_DTYPE, "Lanczos needs FP64 values");
    xab_eig_info loc{};
    xab_eig_info &inf = info ? *info : loc;
    inf = xab_eig_info{};
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    Work W;
    int s;
    if ((s = alloc_work(ctx, W, n, mc)) != XAB_OK) return s;
    const int nb = xab::kRedBlocks;
    hipStream_t st = ctx->stream;
    auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    // q_0 = v0 / ||v0||
    double *sc0 = W.coef;  // first slot, free until the first step
    if ((s = xab::mdot<double>(ctx, nullptr, 0, 0, d_v0, n, W.part, nb, nullptr)) != XAB_OK) return s;
    if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, 1, sc0, 0, nullptr)) != XAB_OK) return s;
    if ((s = xab::scale_precond<double>(ctx, d_v0, sc0, W.V, nullptr, nullptr, n)) != XAB_OK) return s;
    double v0n2 = 0.0;
    XAB_HIP(ctx, hipMemcpyAsync(&v0n2, sc0, sizeof(double), hipMemcpyDeviceToHost, st));
    XAB_HIP(ctx, hipStreamSynchronize(st));
    if (!(v0n2 > 0.0)) return xab_fail(ctx, XAB_E_SHAPE, "start vector is zero");

    const int64_t maxiter = opts->maxiter > 0 ? opts->maxiter : INT64_MAX;
    const int which = opts->which;
    std::vector<double> T((size_t)mc * mc, 0.0);  // row-major projected matrix, stride mc
    std::vector<double> theta, Z, Yc, samples;  // samples: worst wanted estimate / anrm per cycle
    std::vector<int> order(mc);
    int k = 0;  // kept Ritz vectors
    double anrm = 0.0, tscale = 0.0, beta = 0.0;
    int mm = m, status = XAB_NOT_CONVERGED;
    // accuracy policy: the threshold the estimates are held to, narrowed
    // tenfold whenever the true residuals do not confirm a convergence
    double tol_eff = opts->tol;
    int narrowed = 0;
    for (;;) {
        // ---- m - k Lanczos steps, no host round trip
        for (int j = k; j < m; ++j)
            if ((s = recurrence_step(ctx, pl, W, j, mc, n)) != XAB_OK) return s;
        inf.iters += m - k;
        // ---- one read-back of every step's coefficients
        XAB_HIP(ctx, hipMemcpyAsync(W.host, W.coef, W.host_bytes, hipMemcpyDeviceToHost, st));
        XAB_HIP(ctx, hipStreamSynchronize(st));
        const int *gates = (const int *)((const char *)W.host + sizeof(double) * (size_t)W.ld * mc);
        mm = m;
        beta = 0.0;
        for (int j = k; j < m; ++j) {
            const double *h1 = W.host + (size_t)j * W.ld, *h2 = h1 + (mc + 2), *sc = h2 + (mc + 2);
            const bool g = gates[j] != 0;
            const double alpha = h1[j] + (g ? h2[j] : 0.0);
            beta = std::sqrt(g ? sc[0] : h2[j + 1]);
            T[(size_t)j * mc + j] = alpha;
            tscale = std::max({tscale, std::fabs(alpha), beta});
            if (beta <= 1e-14 * tscale) {  // invariant subspace: the cycle ends here
                beta = 0.0;
                mm = j + 1;
                break;
            }
            if (j + 1 < m) T[(size_t)(j + 1) * mc + j] = T[(size_t)j * mc + j + 1] = beta;
        }
        // ---- Ritz pairs of T[:mm, :mm], wanted end first
        std::vector<double> a((size_t)mm * mm);
        for (int i = 0; i < mm; ++i)
            for (int j = 0; j < mm; ++j) a[(size_t)i * mm + j] = T[(size_t)i * mc + j];
        jacobi_eig(mm, a, theta, Z);
        order.resize(mm);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int p, int q) {
            return which == XAB_EIG_LARGEST ? theta[p] > theta[q] : theta[p] < theta[q];
        });
        std::vector<double> th(mm), last(mm);
        for (int i = 0; i < mm; ++i) {
            th[i] = theta[order[i]];
            last[i] = Z[(size_t)(mm - 1) * mm + order[i]];
            anrm = std::max(anrm, std::fabs(th[i]));
        }
        tscale = std::max(tscale, anrm);
        inf.m_final = m;
        {
            double worst = 0.0;
            for (int i = 0; i < std::min(nev, mm); ++i) worst = std::max(worst, std::fabs(beta * last[i]));
            samples.push_back(anrm > 0.0 ? worst / anrm : 0.0);
        }
        int nconv = 0;
        for (int i = 0; i < std::min(nev, mm); ++i)
            if (std::fabs(beta * last[i]) <= tol_eff * anrm) ++nconv;
        inf.nconv = nconv;
        // column-major Y (mm x c) of the first c wanted Ritz vectors
        auto ritz = [&](int c) {
            Yc.assign((size_t)mm * c, 0.0);
            for (int q = 0; q < c; ++q)
                for (int j = 0; j < mm; ++j) Yc[(size_t)q * mm + j] = Z[(size_t)j * mm + order[q]];
        };
        bool done = false;
        if (mm < nev) {
            status = XAB_BREAKDOWN;
            done = true;
        } else if (nconv == nev || beta == 0.0) {
            status = XAB_OK;
            inf.nconv = nev;
            done = true;
        } else if (inf.iters >= maxiter) {
            done = true;
        } else if (opts->max_time_s > 0 && elapsed() > opts->max_time_s) {
            status = XAB_TIME_LIMIT;
            done = true;
        }
        if (done) {
            const int nret = std::min(nev, mm);
            for (int i = 0; i < nev; ++i) h_evals[i] = i < nret ? th[i] : 0.0;
            ritz(nret);
            if ((s = rotate(ctx, W, mm, Yc, nret, d_evecs, n, n)) != XAB_OK) return s;
            // true residual norms ||A x_i - theta_i x_i||
            double worst = 0.0;
            for (int i = 0; i < nret; ++i) {
                const double *xi = d_evecs + (int64_t)i * n;
                if ((s = xab_spmv_dispatch(ctx, pl, xi, XAB_F64, W.w, XAB_F64, XAB_F64)) != XAB_OK) return s;
                hipLaunchKernelGGL(k_eig_resid, dim3(nb), dim3(kRotNT), 0, st, W.w, xi, th[i], nullptr, 0.0, n,
                                   W.part);
                XAB_LAUNCH_CHECK(ctx, "k_eig_resid");
                if ((s = xab::reduce_parts(ctx, W.part, nb, 1, 1, W.coef + i, 0, nullptr)) != XAB_OK) return s;
            }
            XAB_HIP(ctx, hipMemcpyAsync(W.host, W.coef, sizeof(double) * nret, hipMemcpyDeviceToHost, st));
            XAB_HIP(ctx, hipStreamSynchronize(st));
            for (int i = 0; i < nret; ++i) worst = std::max(worst, std::sqrt(W.host[i]));
            inf.anrm = anrm;
            inf.max_resid = anrm > 0.0 ? worst / anrm : worst;
            inf.nret = std::min(nev, mm);
            inf.seconds = elapsed();
            inf.faults = narrowed;
            bool retry = false;
            if (ctx->policy == XAB_ACCURACY && status == XAB_OK && inf.max_resid > opts->tol) {
                // section 3.3.2: the estimates met the threshold, the true
                // residuals do not meet tol: run on with a narrower threshold
                // while the limits allow, else report no convergence
                const bool by_estimate = nconv == nev && beta != 0.0;
                if (by_estimate && narrowed < kMaxNarrowEig && inf.iters < maxiter &&
                    !(opts->max_time_s > 0 && elapsed() > opts->max_time_s)) {
                    tol_eff /= 10.0;
                    inf.faults = ++narrowed;
                    retry = true;
                }
                status = XAB_NOT_CONVERGED;
            }
            if (!retry) {
                inf.status = status;
                return status;
            }
        }
        // ---- thick restart: keep k Ritz vectors (count from the cycle just
        // ended), then q_mm as vector k
        k = nev + (m - nev) / 2;
        ritz(k);
        if ((s = rotate(ctx, W, mm, Yc, k, W.V2, W.ldv, n)) != XAB_OK) return s;
        XAB_HIP(ctx, hipMemcpyAsync(W.V2 + (int64_t)k * W.ldv, W.V + (int64_t)mm * W.ldv, sizeof(double) * n,
                                    hipMemcpyDeviceToDevice, st));
        std::swap(W.V, W.V2);
        std::fill(T.begin(), T.end(), 0.0);
        for (int i = 0; i < k; ++i) {
            T[(size_t)i * mc + i] = th[i];
            T[(size_t)k * mc + i] = T[(size_t)i * mc + k] = beta * last[i];
        }
        inf.restarts++;
        // restart-length judgment (eq. (1)) on the samples since m last changed
        if (tune && m < mc && (int)samples.size() >= window &&
            mm_ratio(samples, samples.size(), window) < opts->mm_ratio) {
            m = std::min(m + opts->restart_step, mc);
            samples.clear();
        }
    }
}
