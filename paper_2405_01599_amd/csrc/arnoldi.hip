// Restarted Arnoldi for the unsymmetric standard eigenproblem (the solver
// list of section 2.2; section 4.3: 10 eigenpairs to 1e-8; section 4.4.2
// tunes its restart frequency).  The restart is the implicit one of
// Sorensen (1992) with exact shifts: after m basis vectors the Ritz values
// of the Hessenberg H = V^T A V are split into the k wanted and m - k
// unwanted ones, the unwanted ones are applied to H as implicit QR shifts
// (a complex pair as one double-shift step), and the first k rotated basis
// vectors plus the new residual direction continue the recurrence, so the
// kept space is the Krylov space filtered by the polynomial whose roots
// are the unwanted Ritz values.
//
// Device side: the same recurrence step as the Lanczos driver (products
// through the plan, classical Gram-Schmidt with the DGKS second pass,
// coefficients in device slots, no host round trip inside a cycle).  Host
// side, once per cycle: the real Schur form of H (Francis double-shift QR),
// Ritz vectors by back substitution for the residual estimates, the shifted
// QR steps, and one basis rotation kernel for the restart.
#include "dense_eig.h"
#include "eig_common.h"

namespace {

using xab::dense::cplx;

struct Ritz {
    cplx lam;
    int pos;  // diagonal position in the Schur form (the block's first row for a pair)
};

double want_key(cplx l, int which) {
    if (which == XAB_EIG_LARGEST) return -l.real();
    if (which == XAB_EIG_SMALLEST) return l.real();
    return -std::abs(l);
}

// Ritz values of the Schur form (wr, wi, diagonal order) sorted wanted-first;
// a pair as (+im, -im), both members pointing at the block's first row.
std::vector<Ritz> sorted_ritz(const std::vector<double> &wr, const std::vector<double> &wi, int which) {
    std::vector<Ritz> r;
    const int n = (int)wr.size();
    for (int p = 0; p < n; ++p) {
        if (wi[p] > 0.0) {
            r.push_back({cplx(wr[p], wi[p]), p});
            r.push_back({cplx(wr[p], -wi[p]), p});
            ++p;
        } else {
            r.push_back({cplx(wr[p], 0.0), p});
        }
    }
    std::stable_sort(r.begin(), r.end(), [&](const Ritz &a, const Ritz &b) {
        const double ka = want_key(a.lam, which), kb = want_key(b.lam, which);
        if (ka != kb) return ka < kb;
        return a.lam.imag() > b.lam.imag();  // a pair: +im first
    });
    return r;
}

// true when entries i-1 and i of the sorted list are the two members of one pair
bool splits_pair(const std::vector<Ritz> &r, int i) {
    return i > 0 && i < (int)r.size() && r[i].lam.imag() != 0.0 && r[i].pos == r[i - 1].pos;
}

}  // namespace

extern "C" int xab_arnoldi(xab_ctx *ctx, const xab_plan *pl, const double *d_v0, const xab_eig_opts *opts,
                           double *h_re, double *h_im, double *d_evecs, xab_eig_info *info) {
    if (!ctx || !pl || !d_v0 || !opts) return XAB_E_NULL;
    const xab_matrix *A = pl->A;
    const int64_t n = A->n;
    const int nev = opts->nev;
    int m = opts->m;
    const bool tune = opts->restart_step > 0 && ctx->policy != XAB_MEMORY;  // MEMORY: the basis keeps its size
    const int mc = tune ? opts->m_max : m;
    const int window = opts->window > 0 ? opts->window : 5;
    if (A->n != A->ncols) return xab_fail(ctx, XAB_E_SHAPE, "Arnoldi needs a square matrix");
    if (nev < 1 || m < nev + 2 || m > kMaxM || m > n)
        return xab_fail(ctx, XAB_E_SHAPE, "need 1 <= nev, nev + 2 <= m <= min(63, n) (nev %d, m %d, n %lld)", nev,
                        m, (long long)n);
    if (tune && (mc < m || mc > kMaxM || mc > n))
        return xab_fail(ctx, XAB_E_SHAPE, "m_max must be in [m, min(63, n)] (m_max %d)", mc);
    if (opts->which != XAB_EIG_LARGEST && opts->which != XAB_EIG_SMALLEST && opts->which != XAB_EIG_MAGNITUDE)
        return xab_fail(ctx, XAB_E_SHAPE, "which");
    if (!h_re || !h_im || !d_evecs) return XAB_E_NULL;
    if (!A->has64) return xab_fail(ctx, XAB_E_DTYPE, "Arnoldi needs FP64 values");
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
    double v0n = 0.0;
    if ((s = device_norm(ctx, W, d_v0, n, &v0n)) != XAB_OK) return s;
    if (!(v0n > 0.0)) return xab_fail(ctx, XAB_E_SHAPE, "start vector is zero");
    if ((s = xab::scale_from<double, double>(ctx, d_v0, 1.0 / v0n, W.V, nullptr, nullptr, n)) != XAB_OK) return s;

    const int64_t maxiter = opts->maxiter > 0 ? opts->maxiter : INT64_MAX;
    const int which = opts->which;
    std::vector<double> H((size_t)(mc + 1) * mc, 0.0);  // row-major, stride mc
    std::vector<double> samples, Ycm;
    int k = 0;
    double anrm = 0.0, tscale = 0.0;
    // accuracy policy: the threshold the estimates are held to, narrowed
    // tenfold whenever the true residuals do not confirm a convergence
    double tol_eff = opts->tol;
    int narrowed = 0;
    for (;;) {
        // ---- m - k recurrence steps, no host round trip
        for (int j = k; j < m; ++j)
            if ((s = recurrence_step(ctx, pl, W, j, mc, n)) != XAB_OK) return s;
        inf.iters += m - k;
        XAB_HIP(ctx, hipMemcpyAsync(W.host, W.coef, W.host_bytes, hipMemcpyDeviceToHost, st));
        XAB_HIP(ctx, hipStreamSynchronize(st));
        const int *gates = (const int *)((const char *)W.host + sizeof(double) * (size_t)W.ld * mc);
        int mm = m;
        double beta = 0.0;
        for (int j = k; j < m; ++j) {
            const double *h1 = W.host + (size_t)j * W.ld, *h2 = h1 + (mc + 2), *sc = h2 + (mc + 2);
            const bool g = gates[j] != 0;
            for (int i = 0; i <= j; ++i) {
                H[(size_t)i * mc + j] = h1[i] + (g ? h2[i] : 0.0);
                tscale = std::max(tscale, std::fabs(H[(size_t)i * mc + j]));
            }
            beta = std::sqrt(g ? sc[0] : h2[j + 1]);
            tscale = std::max(tscale, beta);
            if (beta <= 1e-14 * tscale) {  // invariant subspace
                beta = 0.0;
                mm = j + 1;
                break;
            }
            H[(size_t)(j + 1) * mc + j] = beta;
        }
        // ---- Ritz values (real Schur form of H[:mm, :mm]) and estimates
        std::vector<double> T((size_t)mm * mm), Z((size_t)mm * mm, 0.0), wr, wi;
        for (int i = 0; i < mm; ++i) {
            for (int j = 0; j < mm; ++j) T[(size_t)i * mm + j] = i <= j + 1 ? H[(size_t)i * mc + j] : 0.0;
            Z[(size_t)i * mm + i] = 1.0;
        }
        if (!xab::dense::schur(mm, T, Z, wr, wi))
            return xab_fail(ctx, XAB_E_DEVICE, "Arnoldi: the QR iteration on the projected matrix did not converge");
        const std::vector<Ritz> R = sorted_ritz(wr, wi, which);
        for (const Ritz &r : R) anrm = std::max(anrm, std::abs(r.lam));
        tscale = std::max(tscale, anrm);
        int ne = std::min(nev, mm);
        if (splits_pair(R, ne)) ++ne;
        // Ritz vectors y = Z x (complex, ||y|| = 1) of the first ne values
        std::vector<std::vector<cplx>> Y(ne);
        std::vector<double> est(ne, 0.0);
        for (int i = 0; i < ne; ++i) {
            if (i > 0 && R[i].pos == R[i - 1].pos) {  // conjugate of the previous one
                Y[i] = Y[i - 1];
                for (cplx &v : Y[i]) v = std::conj(v);
                est[i] = est[i - 1];
                continue;
            }
            std::vector<cplx> x;
            xab::dense::ritz_vec(mm, T, R[i].pos, x);
            std::vector<cplx> y(mm, cplx(0.0, 0.0));
            for (int r = 0; r < mm; ++r)
                for (int c = 0; c < mm; ++c) y[r] += Z[(size_t)r * mm + c] * x[c];
            double nr = 0.0;
            for (const cplx &v : y) nr += std::norm(v);
            nr = std::sqrt(nr);
            for (cplx &v : y) v /= nr;
            Y[i] = y;
            est[i] = std::fabs(beta) * std::abs(y[mm - 1]);
        }
        int nconv = 0;
        double worst = 0.0;
        for (int i = 0; i < ne; ++i) {
            worst = std::max(worst, est[i]);
            if (est[i] <= tol_eff * anrm) ++nconv;
        }
        samples.push_back(anrm > 0.0 ? worst / anrm : 0.0);
        inf.nconv = nconv;
        inf.m_final = m;
        bool done = false;
        int status = XAB_NOT_CONVERGED;
        if (mm < nev) {
            status = XAB_BREAKDOWN;
            done = true;
        } else if (nconv == ne || beta == 0.0) {
            status = XAB_OK;
            inf.nconv = ne;
            done = true;
        } else if (inf.iters >= maxiter) {
            done = true;
        } else if (opts->max_time_s > 0 && elapsed() > opts->max_time_s) {
            status = XAB_TIME_LIMIT;
            done = true;
        }
        if (done) {
            // eigenvalues and vectors, a pair as real and imaginary parts (dgeev's layout)
            for (int i = 0; i <= nev; ++i) {
                h_re[i] = i < ne ? R[i].lam.real() : 0.0;
                h_im[i] = i < ne ? R[i].lam.imag() : 0.0;
            }
            Ycm.assign((size_t)mm * ne, 0.0);
            for (int i = 0; i < ne; ++i)
                for (int r = 0; r < mm; ++r)
                    Ycm[(size_t)i * mm + r] =
                        (i > 0 && R[i].pos == R[i - 1].pos) ? Y[i - 1][r].imag() : Y[i][r].real();
            if ((s = rotate(ctx, W, mm, Ycm, ne, d_evecs, n, n)) != XAB_OK) return s;
            // true residuals: ||A x - lam x||, a pair over both parts
            int slot = 0;
            for (int i = 0; i < ne; ++i) {
                const double *xi = d_evecs + (int64_t)i * n;
                const bool first = R[i].lam.imag() != 0.0 && !(i > 0 && R[i].pos == R[i - 1].pos);
                const bool second = i > 0 && R[i].pos == R[i - 1].pos;
                const double lr = R[i].lam.real(), li = std::fabs(R[i].lam.imag());
                if ((s = xab_spmv_dispatch(ctx, pl, xi, XAB_F64, W.w, XAB_F64, XAB_F64)) != XAB_OK) return s;
                if (first)  // A x_re - lr x_re + li x_im
                    hipLaunchKernelGGL(k_eig_resid, dim3(nb), dim3(kRotNT), 0, st, W.w, xi, lr, xi + n, -li, n,
                                       W.part);
                else if (second)  // A x_im - lr x_im - li x_re
                    hipLaunchKernelGGL(k_eig_resid, dim3(nb), dim3(kRotNT), 0, st, W.w, xi, lr, xi - n, li, n,
                                       W.part);
                else
                    hipLaunchKernelGGL(k_eig_resid, dim3(nb), dim3(kRotNT), 0, st, W.w, xi, lr, nullptr, 0.0, n,
                                       W.part);
                XAB_LAUNCH_CHECK(ctx, "k_eig_resid");
                if ((s = xab::reduce_parts(ctx, W.part, nb, 1, 1, W.coef + 1 + slot++, 0, nullptr)) != XAB_OK)
                    return s;
            }
            XAB_HIP(ctx, hipMemcpyAsync(W.host, W.coef + 1, sizeof(double) * ne, hipMemcpyDeviceToHost, st));
            XAB_HIP(ctx, hipStreamSynchronize(st));
            double wres = 0.0;
            for (int i = 0; i < ne; ++i) {
                const bool first = R[i].lam.imag() != 0.0 && !(i > 0 && R[i].pos == R[i - 1].pos);
                const double r2 = first && i + 1 < ne ? W.host[i] + W.host[i + 1] : W.host[i];
                if (first && i + 1 < ne) {
                    wres = std::max(wres, std::sqrt(r2));
                    ++i;
                } else {
                    wres = std::max(wres, std::sqrt(r2));
                }
            }
            inf.anrm = anrm;
            inf.max_resid = anrm > 0.0 ? wres / anrm : wres;
            inf.nret = ne;
            inf.seconds = elapsed();
            inf.faults = narrowed;
            bool retry = false;
            if (ctx->policy == XAB_ACCURACY && status == XAB_OK && inf.max_resid > opts->tol) {
                // section 3.3.2: the estimates met the threshold, the true
                // residuals do not meet tol: run on with a narrower threshold
                // while the limits allow, else report no convergence
                const bool by_estimate = nconv == ne && beta != 0.0;
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
        // ---- implicit restart with the unwanted Ritz values as exact shifts
        int kk = nev + (m - nev) / 2;
        if (splits_pair(R, kk)) kk = kk + 1 < m ? kk + 1 : kk - 1;
        std::vector<double> Hs((size_t)mm * mm), Q((size_t)mm * mm, 0.0);
        for (int i = 0; i < mm; ++i) {
            for (int j = 0; j < mm; ++j) Hs[(size_t)i * mm + j] = i <= j + 1 ? H[(size_t)i * mc + j] : 0.0;
            Q[(size_t)i * mm + i] = 1.0;
        }
        for (int i = kk; i < mm; ++i) {
            const cplx mu = R[i].lam;
            if (mu.imag() == 0.0) {
                xab::dense::qr_shift1(mm, Hs, Q, mu.real());
            } else {  // a pair (kk never splits one): one double-shift step, then skip the partner
                xab::dense::qr_shift2(mm, Hs, Q, 2.0 * mu.real(), std::norm(mu));
                if (i + 1 < mm && R[i + 1].pos == R[i].pos) ++i;
            }
        }
        // new basis: v+_c = V Q[:, c] (c < kk) and the residual direction
        // f = V Q[:, kk] * H+[kk, kk-1] + v_mm * beta * Q[mm-1, kk-1]
        Ycm.assign((size_t)(mm + 1) * (kk + 1), 0.0);
        for (int c = 0; c < kk; ++c)
            for (int r = 0; r < mm; ++r) Ycm[(size_t)c * (mm + 1) + r] = Q[(size_t)r * mm + c];
        const double hk = Hs[(size_t)kk * mm + kk - 1];
        for (int r = 0; r < mm; ++r) Ycm[(size_t)kk * (mm + 1) + r] = hk * Q[(size_t)r * mm + kk];
        Ycm[(size_t)kk * (mm + 1) + mm] = beta * Q[(size_t)(mm - 1) * mm + kk - 1];
        if ((s = rotate(ctx, W, mm + 1, Ycm, kk + 1, W.V2, W.ldv, n)) != XAB_OK) return s;
        std::swap(W.V, W.V2);
        double *vk = W.V + (int64_t)kk * W.ldv;
        double bk = 0.0;
        if ((s = device_norm(ctx, W, vk, n, &bk)) != XAB_OK) return s;
        std::fill(H.begin(), H.end(), 0.0);
        for (int i = 0; i < kk; ++i)
            for (int j = 0; j < kk; ++j) H[(size_t)i * mc + j] = i <= j + 1 ? Hs[(size_t)i * mm + j] : 0.0;
        inf.restarts++;
        if (bk <= 1e-14 * tscale) {
            // the kept space is invariant: its Ritz pairs are exact; one more
            // evaluation with no new steps ends the solve
            k = kk;
            m = kk;
            continue;
        }
        if ((s = xab::scale_from<double, double>(ctx, vk, 1.0 / bk, vk, nullptr, nullptr, n)) != XAB_OK) return s;
        H[(size_t)kk * mc + kk - 1] = bk;
        k = kk;
        if (tune && m < mc && (int)samples.size() >= window &&
            mm_ratio(samples, samples.size(), window) < opts->mm_ratio) {
            m = std::min(m + opts->restart_step, mc);
            samples.clear();
        }
    }
}
