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
//
// The Hessenberg column, the Givens rotations and the residual recurrence
// of each Arnoldi step run on the device (one small kernel at the end of
// the step), so a cycle's steps are queued back to back: the host never
// waits for the step the GPU is running.  It waits for the step before
// that one (to stop queueing once a step has met the threshold or broken
// down), and for the running step too only when the recurrence is about
// to meet the threshold, by reading the step counter the step kernel
// publishes in coherent host memory: no marker packet sits between two
// steps on the stream.  A step queued after the stopping one computes
// into the next basis slot and leaves the rotated system alone.  The host
// reads the rotated system back once per cycle.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "blas.h"

namespace {

constexpr double kEta = 0.70710678118654752440;  // DGKS threshold 1/sqrt(2)

// What the step kernel leaves where the host can read it without a copy
// (coherent pinned memory): the last step done, the stop flag and the
// recurrence residuals |g_0| .. |g_k|.
struct Mirror {
    int done;
    int k;
    int stop;
    int breakdown;
    int by_rec;
    double absg[64];
};

// Device state of one cycle: the rotated Hessenberg matrix (row i, column
// j at H[i ld + j]), the rotations, the rotated right-hand side g.
struct CycleState {
    int k;
    int stop;
    double tol_abs;
};

struct Work {
    xab_ctx *ctx = nullptr;
    void *base = nullptr;
    double *r = nullptr;     // FP64 residual / product buffer [n]
    double *part = nullptr;  // partial sums [kRedBlocks * kPartLd]
    double *h1 = nullptr, *h2 = nullptr, *sc = nullptr;  // small device vectors
    int *gate = nullptr;
    void *V = nullptr, *w = nullptr, *z = nullptr;
    int64_t ldv = 0;
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;  // rotated system (device)
    CycleState *st = nullptr;
    size_t sys_bytes = 0;    // H .. g, read back once per cycle
    double *host = nullptr;  // pinned: the rotated system's read-back, then y
    Mirror *mir = nullptr;   // coherent pinned, written by the step kernel
    Mirror *mir_dev = nullptr;
    ~Work() {
        if (base) xab_dfree(ctx, base);
        if (host) (void)hipHostFree(host);
        if (mir) (void)hipHostFree(mir);
    }
};

// The end of Arnoldi step j in one launch.  Every workgroup but the last
// forms 256 rows of v_{j+1} = w / ||w|| and z = M^-1 v_{j+1} (the squared
// norm h2[j+1], or sc when the DGKS gate fired; h1[j+1] without DGKS).
// The last workgroup takes the step's Hessenberg column (h1, plus h2 when
// the gate fired) and its norm, applies the earlier rotations to it, forms
// the rotation that zeroes h_{j+1,j}, updates g and decides whether the
// cycle stops (breakdown, or |g_{j+1}| at the threshold): its lanes stage
// the column and the rotations in LDS and lane 0 runs the chain of at most
// 63 rotations, row i + 1 carried in a register.
template <class T>
__global__ __launch_bounds__(256) void k_gmres_step_end(int j, int ld, int dgks, const double *__restrict__ h1,
                                                        const double *__restrict__ h2, const double *__restrict__ sc,
                                                        const int *__restrict__ gate_p, const T *__restrict__ w,
                                                        T *__restrict__ v, T *__restrict__ z, const T *__restrict__ d,
                                                        int64_t n, int nblk, double *__restrict__ H,
                                                        double *__restrict__ cs, double *__restrict__ sn,
                                                        double *__restrict__ g, CycleState *__restrict__ st,
                                                        Mirror *mir) {
    const int t = threadIdx.x;
    if ((int)blockIdx.x < nblk) {
        const int64_t r = (int64_t)blockIdx.x * 256 + t;
        if (r < n) {
            if (dgks) xab::scale_precond_row(w, h2 + j + 1, sc, gate_p, v, z, d, r);
            else xab::scale_precond_row<T>(w, h1 + j + 1, nullptr, nullptr, v, z, d, r);
        }
        return;
    }
    __shared__ double col[64], rc[64], rs[64];
    if (st->stop) {
        // queued after the stopping step: leave the rotated system alone
        if (t == 0) mir->done = j;
        return;
    }
    const int gate = dgks ? *gate_p : 0;
    if (t <= j) col[t] = h1[t] + (gate ? h2[t] : 0.0);
    if (t < j) {
        rc[t] = cs[t];
        rs[t] = sn[t];
    }
    __syncthreads();
    if (t == 0) {
        const double hn = sqrt(!dgks ? h1[j + 1] : (gate ? sc[0] : h2[j + 1]));
        double cur = col[0];  // row i of the column after rotations 0 .. i - 1
        for (int i = 0; i < j; ++i) {
            const double a = cur, c = col[i + 1];
            col[i] = rc[i] * a + rs[i] * c;
            cur = -rs[i] * a + rc[i] * c;
        }
        const double rr = hypot(cur, hn);
        const double cj = rr == 0.0 ? 1.0 : cur / rr, sj = rr == 0.0 ? 0.0 : hn / rr;
        cs[j] = cj;
        sn[j] = sj;
        col[j] = rr;
        H[(size_t)(j + 1) * ld + j] = 0.0;
        const double gj = g[j];
        g[j + 1] = -sj * gj;
        g[j] = cj * gj;
        st->k = j + 1;
        mir->k = j + 1;
        const double ag = fabs(sj * gj);
        const int brk = hn == 0.0, rec = !brk && ag <= st->tol_abs;
        st->stop = brk || rec;
        mir->absg[j + 1] = ag;
        mir->breakdown = brk;
        mir->by_rec = rec;
        mir->stop = brk || rec;
    }
    __syncthreads();
    if (t <= j) H[(size_t)t * ld + j] = col[t];
    if (t == 0) {
        __threadfence_system();
        mir->done = j;
    }
}

__global__ void k_gmres_cycle_init(double beta, double tol_abs, double *__restrict__ g, CycleState *__restrict__ st) {
    if (threadIdx.x != 0) return;
    g[0] = beta;
    st->k = 0;
    st->stop = 0;
    st->tol_abs = tol_abs;
}

int alloc_work(xab_ctx *ctx, Work &W, int64_t n, int m, size_t tsize) {
    W.ctx = ctx;
    W.ldv = (n + 63) / 64 * 64;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off_r = 0, off_part = off_r + al(sizeof(double) * n);
    size_t off_small = off_part + al(sizeof(double) * xab::kRedBlocks * xab::kPartLd);
    size_t off_sys = off_small + al(sizeof(double) * (3 * (m + 2) + 16) + 64);
    size_t sys_bytes = sizeof(double) * ((size_t)(m + 1) * m + 2 * (size_t)m + (m + 1));
    size_t off_st = off_sys + al(sys_bytes);
    size_t off_V = off_st + al(sizeof(CycleState));
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
    W.H = (double *)(b + off_sys);
    W.cs = W.H + (size_t)(m + 1) * m;
    W.sn = W.cs + m;
    W.g = W.sn + m;
    W.sys_bytes = sys_bytes;
    W.st = (CycleState *)(b + off_st);
    if (hipHostMalloc((void **)&W.host, sys_bytes, hipHostMallocDefault) != hipSuccess) {
        W.host = nullptr;
        return xab_fail(ctx, XAB_E_NOMEM, "pinned host buffer");
    }
    if (hipHostMalloc((void **)&W.mir, sizeof(Mirror), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        W.mir = nullptr;
        return xab_fail(ctx, XAB_E_NOMEM, "pinned host buffer");
    }
    if (hipHostGetDevicePointer((void **)&W.mir_dev, W.mir, 0) != hipSuccess)
        return xab_fail(ctx, XAB_E_DEVICE, "device address of the step mirror");
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
    if (m > 63) return xab_fail(ctx, XAB_E_SHAPE, "restart length above 63");
    Mirror *mir = W.mir;
    mir->done = -1;
    mir->k = 0;
    mir->stop = 0;
    mir->breakdown = 0;
    mir->by_rec = 0;
    mir->absg[0] = beta;
    hipLaunchKernelGGL(k_gmres_cycle_init, dim3(1), dim3(64), 0, ctx->stream, beta, tol_abs, W.g, W.st);
    XAB_LAUNCH_CHECK(ctx, "k_gmres_cycle_init");
    out.breakdown = false;
    // until step q's kernel has published its rotation: a spin on the
    // counter in coherent host memory; a step that has not reported within
    // the spin limit (20 ms, or XAB_STEP_WAIT_MS; a very large matrix, or a
    // failed launch) is waited for by draining the stream, which also
    // returns any error of the queued work
    const char *wenv = getenv("XAB_STEP_WAIT_MS");
    const long wait_ms = wenv && *wenv ? std::max(0L, strtol(wenv, nullptr, 10)) : 20L;
    auto wait_step = [&](int q) -> int {
        const volatile int *done = &mir->done;
        if (*done < q) {
            const auto t0 = std::chrono::steady_clock::now();
            while (*done < q) {
                if (std::chrono::steady_clock::now() - t0 >= std::chrono::milliseconds(wait_ms)) {
                    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
                    break;
                }
#if defined(__x86_64__)
                __builtin_ia32_pause();
#endif
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);  // no read of the mirror moves above the wait
        return XAB_OK;
    };
    for (int j = 0; j < m && j < max_steps; ++j) {
        if (j >= 2) {
            // the GPU is on step j - 1 (or earlier): stop queueing once a
            // finished step has stopped the cycle
            if ((s = wait_step(j - 2)) != XAB_OK) return s;
            if (mir->stop) break;
            // the recurrence near the threshold: let step j - 1 finish too
            // rather than queue a step past the stop
            const double a = mir->absg[j - 1], b = mir->absg[j - 2];
            const double pred = b > 0.0 ? a * std::min(1.0, a / b) : 0.0;
            if (pred <= 100.0 * tol_abs) {
                if ((s = wait_step(j - 1)) != XAB_OK) return s;
                if (mir->stop) break;
            }
        }
        // w = A z (FP64 accumulation in every mode)
        if ((s = xab_spmv_dispatch(ctx, pl, z, tt, w, tt, XAB_F64)) != XAB_OK) return s;
        bool dgks = false;
        if (ortho == XAB_ORTHO_DGKS) {
            // pass 1: h1 = V^T w, ||w||^2; then one sweep: w' = w - V h1 with
            // the second pass's h2 = V^T w', ||w'||^2 from the same reads of V
            dgks = true;
            if ((s = xab::mdot<T>(ctx, V, W.ldv, j + 1, w, n, W.part, nb, nullptr)) != XAB_OK) return s;
            if ((s = xab::reduce_parts(ctx, W.part, nb, xab::kPartLd, j + 2, W.h1, 0, nullptr)) != XAB_OK) return s;
            if ((s = xab::update_mdot<T>(ctx, V, j + 1, W.h1, V, j + 1, W.ldv, w, n, W.part, nb)) != XAB_OK) return s;
            // h2 and the DGKS decision: the second update only when
            // cancellation was severe
            if ((s = xab::reduce_parts_dgks(ctx, W.part, nb, xab::kPartLd, j + 2, W.h2, W.h1 + j + 1, kEta, W.gate)) !=
                XAB_OK)
                return s;
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
        // v_{j+1} = w / ||w||, z = M^-1 v_{j+1}, and the step's rotation
        T *vn = V + (int64_t)(j + 1) * W.ldv;
        const int nblk = (int)((n + 255) / 256);
        hipLaunchKernelGGL((k_gmres_step_end<T>), dim3((unsigned)nblk + 1), dim3(256), 0, ctx->stream, j, m,
                           dgks ? 1 : 0, W.h1, W.h2, W.sc, W.gate, w, vn, z, d, n, nblk, W.H, W.cs, W.sn, W.g, W.st,
                           W.mir_dev);
        XAB_LAUNCH_CHECK(ctx, "k_gmres_step_end");
    }
    // one read-back of the rotated system per cycle
    XAB_HIP(ctx, hipMemcpyAsync(W.host, W.H, W.sys_bytes, hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int k = mir->k;  // steps before the stop (steps queued after it left no trace)
    const double *H = W.host, *g = W.host + (W.g - W.H);
    out.samp.assign(mir->absg, mir->absg + k + 1);
    out.breakdown = mir->breakdown != 0;
    out.by_recurrence = mir->by_rec != 0;
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
        // y through the pinned buffer (the rotated system there is consumed)
        std::copy(y.begin(), y.end(), W.host);
        XAB_HIP(ctx, hipMemcpyAsync(W.h2, W.host, sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
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
