// Batched independent systems: the block-diagonal concatenation of many
// CSR matrices, one SpMV launch over all of them, and BiCGStab (van der
// Vorst's form, the paper's second linear solver) advancing every system at
// once.  One iteration is twelve kernels: a work-list kernel (the segments
// and SELL windows of the systems still active), two SpMVs, five row kernels
// over segments of kSegRows rows (a large system spans many workgroups) and
// four one-wave-per-system kernels that sum the segments' partial inner
// products in a fixed order and take the scalar decisions.  It is captured
// once in a HIP graph and replayed.  Per-system scalars live on the device;
// a system that converges (or breaks down) is masked from then on and drops
// out of the next iteration's lists (segmented-scan tiles whose systems are
// all inactive skip their work).  Each system has its own threshold: under
// the accuracy policy a system whose true residual misses tol at the end
// restarts from its x with a tenfold narrower one.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "segchunk.h"
#include "sell_body.h"

namespace {

using xab::Seg;
constexpr int kNT = 256;
constexpr int kBatchJ = 4;  // entries per lane of the batched SpMV tiles
constexpr int kBiNT = 1024; // threads of the set-up / final kernels (one workgroup per system)
constexpr int kSegRows = 1024; // rows of one system per workgroup of the BiCGStab row kernels
constexpr int kVT = 256;      // threads of the BiCGStab row kernels
constexpr int kFT = 256;      // threads of the per-system kernels (one wave per system)
constexpr int kSellSigma = 1024; // sorting window of the sliced ELLPACK copy
constexpr int kMaxNarrow = 8;    // accuracy policy: tenfold narrowings of a system's threshold at most


// Batched SpMV over the concatenation, in segmented-scan tiles of
// kNT * kBatchJ entries (the BSS layout).  A tile whose rows span at most two
// systems, both converged, is skipped: it only marks that it leaves no
// partial row (any row it shares with a neighbouring tile belongs to one of
// those converged systems, whose products are never read).
template <class T>
__global__ __launch_bounds__(kNT) void k_batch_spmv(const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ colind, const T *__restrict__ val,
                                                    const T *__restrict__ x, T *__restrict__ y, int64_t nnz, int64_t P,
                                                    const int32_t *__restrict__ row_lo,
                                                    const int32_t *__restrict__ tile_row,
                                                    const int32_t *__restrict__ carry_row,
                                                    double *__restrict__ carry_val, double *__restrict__ tail_val,
                                                    int32_t *__restrict__ tail_row,
                                                    const int32_t *__restrict__ sys_of_row, int32_t n,
                                                    const int *__restrict__ active) {
    __shared__ int32_t head_row[kNT * kBatchJ];
    __shared__ Seg<double> wave_tot[kNT / xab::kWave];
    const int64_t t = xab::xcd_remap(blockIdx.x, P);
    if (active) {
        const int32_t ra = tile_row[t], rb = tile_row[t + 1] < n ? tile_row[t + 1] : n - 1;
        const int32_t s0 = sys_of_row[ra], s1 = sys_of_row[rb];
        if (s1 - s0 <= 1 && !active[s0] && !active[s1]) {
            if (threadIdx.x == 0) tail_row[t] = -1;
            return;
        }
    }
    xab::bss_tile<kNT, T, T, T, double, kBatchJ>(t, rowptr, colind, val, x, y, nnz, row_lo, carry_row, carry_val,
                                                 tail_val, tail_row, head_row, wave_tot, nullptr);
}

// Batched SpMV over the sliced ELLPACK copy of the concatenation (64 ordered
// rows per chunk, one lane per row, one wave per chunk).  A chunk none of
// whose rows belongs to an active system is skipped (its products are never
// read); otherwise every row of the chunk is computed.
constexpr int kSellC = xab_plan::kSellC;
constexpr int kSellUnroll = 12; // entries per lane in flight: the random-row systems are held by the gather rate

template <class T>
__global__ __launch_bounds__(kNT) void k_batch_sell(const int64_t *__restrict__ cptr, const int32_t *__restrict__ clen,
                                                    const int32_t *__restrict__ rlen, const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ cols, const T *__restrict__ val,
                                                    const T *__restrict__ x, T *__restrict__ y, int32_t n, int64_t nch,
                                                    int64_t nwg, const int32_t *__restrict__ sys_of_row,
                                                    const int *__restrict__ active) {
    const int64_t wg = xab::xcd_remap(blockIdx.x, nwg);
    const int64_t c = wg * (kNT / kSellC) + threadIdx.x / kSellC;
    if (c >= nch) return;
    const int l = threadIdx.x % kSellC;
    const int64_t r = c * kSellC + l;
    const int32_t row = r < n ? perm[r] : -1;
    if (active) {
        const bool mine = row >= 0 && active[sys_of_row[row]] != 0;
        if (__ballot(mine) == 0) return;  // wave-uniform: the wave is the chunk
    }
    const double acc = xab::sell_lane_sum<T, T, double, kSellUnroll>(val, cols, x, cptr[c] + l, clen[c], rlen[r]);
    if (row >= 0) y[row] = (T)acc;
}

// The same SpMV over the windows listed for this iteration (kSellSigma rows:
// kWinItems workgroup items of 4 chunks).  The items are dealt so that each
// XCD serves a contiguous range of them, whatever their number; workgroups
// past the last item return at once.
constexpr int kWinItems = kSellSigma / kSellC / (kNT / kSellC);

template <class T>
__global__ __launch_bounds__(kNT) void k_batch_sell_listed(const int64_t *__restrict__ cptr,
                                                           const int32_t *__restrict__ clen,
                                                           const int32_t *__restrict__ rlen,
                                                           const int32_t *__restrict__ perm,
                                                           const int32_t *__restrict__ cols, const T *__restrict__ val,
                                                           const T *__restrict__ x, T *__restrict__ y, int32_t n,
                                                           int64_t nch, const int32_t *__restrict__ win_list,
                                                           const int *__restrict__ lcount) {
    const int64_t N = (int64_t)lcount[1] * kWinItems;
    const int64_t q = N / xab::kXcds, rem = N % xab::kXcds;
    const int64_t xcd = blockIdx.x % xab::kXcds, slot = blockIdx.x / xab::kXcds;
    if (slot >= q + (xcd < rem ? 1 : 0)) return;
    const int64_t item = xcd * q + (xcd < rem ? xcd : rem) + slot;
    const int64_t c = ((int64_t)win_list[item / kWinItems] * kWinItems + item % kWinItems) * (kNT / kSellC) +
                      threadIdx.x / kSellC;
    if (c >= nch) return;
    const int l = threadIdx.x % kSellC;
    const int64_t r = c * kSellC + l;
    const int32_t row = r < n ? perm[r] : -1;
    const double acc = xab::sell_lane_sum<T, T, double, kSellUnroll>(val, cols, x, cptr[c] + l, clen[c], rlen[r]);
    if (row >= 0) y[row] = (T)acc;
}

// rows cut by a tile end: start partial plus the following tiles' carries,
// in ascending tile order
template <class T>
__global__ void k_batch_fixup(T *__restrict__ y, int64_t P, const int32_t *__restrict__ carry_row,
                              const double *__restrict__ carry_val, const double *__restrict__ tail_val,
                              const int32_t *__restrict__ tail_row) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    const int32_t r = tail_row[t];
    if (r < 0) return;
    double acc = tail_val[t];
    for (int64_t u = t + 1; u < P && carry_row[u] == r; ++u) acc += carry_val[u];
    y[r] = (T)acc;
}

__device__ __forceinline__ double bsum(double v, double *sh) {
    v = xab::wave_sum(v);
    const int w = threadIdx.x / xab::kWave;
    if (threadIdx.x % xab::kWave == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kBiNT / xab::kWave; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Per-system solver state (device).
struct SysState {
    double rho, alpha, omega, beta, bnorm, res;
    int iters, status;  // status: 0 converged, 1 running/not converged, 2 breakdown
};

// ||b||, r = b - A x0 (A x0 given in ax), rhat = r, p = v = 0, rho = <rhat, r>,
// scalars reset (beta = 0 makes the first direction p = r).  With `redo`,
// only the marked systems restart (from their current x, keeping their
// iteration counts): the accuracy policy's second run.
template <class T>
__global__ __launch_bounds__(kBiNT) void k_bi_init(const int64_t *__restrict__ row_off, const T *__restrict__ bvec,
                                                 const T *__restrict__ ax, T *__restrict__ r, T *__restrict__ rh,
                                                 T *__restrict__ p, T *__restrict__ v, SysState *__restrict__ st,
                                                 int *__restrict__ active, int *__restrict__ early,
                                                 const double *__restrict__ tolv, const int *__restrict__ redo,
                                                 int *__restrict__ n_active) {
    __shared__ double sh[kBiNT / xab::kWave];
    const int k = blockIdx.x;
    if (redo && !redo[k]) return;
    const int64_t r0 = row_off[k], r1 = row_off[k + 1];
    double bb = 0.0, rr = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBiNT) {
        double bi = (double)bvec[i];
        T ri = (T)(bi - (double)ax[i]);
        r[i] = ri;
        rh[i] = ri;
        p[i] = T(0);
        v[i] = T(0);
        bb += bi * bi;
        rr += (double)ri * (double)ri;
    }
    bb = bsum(bb, sh);
    rr = bsum(rr, sh);
    if (threadIdx.x == 0) {
        SysState s;
        s.rho = rr;
        s.alpha = 1.0;
        s.omega = 1.0;
        s.beta = 0.0;
        s.bnorm = bb > 0.0 ? sqrt(bb) : 1.0;
        s.res = sqrt(rr) / s.bnorm;
        s.iters = redo ? st[k].iters : 0;
        s.status = s.res <= tolv[k] ? 0 : (rr == 0.0 ? 2 : 1);
        st[k] = s;
        active[k] = s.status == 1;
        early[k] = 0;
        if (s.status == 1) atomicAdd(n_active, 1);
    }
}

// ---- work lists of one iteration: the row segments of the systems active at
// its start and the SELL windows (kSellSigma rows) holding a row of one,
// appended in any order (each item's work does not depend on its place).
// The counts are cleared by the last kernel of the previous iteration.
// Systems that stop during the iteration stay listed; the kernels test
// their masks.
__device__ __forceinline__ void wave_append(bool pred, int32_t item, int32_t *__restrict__ list,
                                            int *__restrict__ count) {
    const unsigned long long bal = __ballot(pred);
    if (bal == 0) return;  // wave-uniform
    const int lane = threadIdx.x % xab::kWave, leader = __ffsll((long long)bal) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(bal));
    base = __shfl(base, leader);
    if (pred) list[base + __popcll(bal & ((1ull << lane) - 1ull))] = item;
}

__global__ __launch_bounds__(256) void k_bi_lists(int64_t n, int64_t nseg, int64_t nwin,
                                                  const int32_t *__restrict__ seg_sys,
                                                  const int32_t *__restrict__ sys_of_row,
                                                  const int *__restrict__ active, int32_t *__restrict__ seg_list,
                                                  int32_t *__restrict__ win_list, int *__restrict__ count) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    wave_append(g < nseg && active[seg_sys[g]] != 0, (int32_t)g, seg_list, &count[0]);
    bool w_on = false;
    if (g < nwin) {
        const int32_t k0 = sys_of_row[g * kSellSigma];
        const int32_t k1 = sys_of_row[min(n, (g + 1) * kSellSigma) - 1];
        for (int32_t k = k0; k <= k1 && !w_on; ++k) w_on = active[k] != 0;
    }
    wave_append(w_on, (int32_t)g, win_list, &count[1]);
}

// ---- row kernels: one workgroup per listed segment of kSegRows rows of one
// system, so that a large system is spread over many CUs.  Each reads the
// scalars of its system (written by the per-system kernels, never by a row
// kernel) and leaves its inner products as one partial per segment.
struct SegRange {
    int k;
    int64_t r0, r1;
};

__device__ __forceinline__ SegRange seg_range(int32_t j, const int32_t *__restrict__ seg_sys,
                                              const int32_t *__restrict__ seg_off,
                                              const int64_t *__restrict__ row_off) {
    const int k = seg_sys[j];
    const int64_t r0 = row_off[k] + (int64_t)(j - seg_off[k]) * kSegRows;
    return {k, r0, min(r0 + (int64_t)kSegRows, row_off[k + 1])};
}

// workgroup sum in a fixed order: xor tree in each wave, then the waves in order
__device__ __forceinline__ double vsum(double v, double *sh) {
    v = xab::wave_sum(v);
    if (threadIdx.x % xab::kWave == 0) sh[threadIdx.x / xab::kWave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kVT / xab::kWave; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// the listed segment of this workgroup (the kernel returns past the list's end)
#define XAB_LISTED_SEGMENT(j)                                \
    if ((int64_t)blockIdx.x >= (int64_t)lcount[0]) return;   \
    const int32_t j = seg_list[blockIdx.x]

#define XAB_SEG_ROWS(R, i)                                              \
    _Pragma("unroll") for (int u_ = 0; u_ < kSegRows / kVT; ++u_)       \
        if (const int64_t i = (R).r0 + threadIdx.x + (int64_t)u_ * kVT; i < (R).r1)

// p = r + beta (p - omega v), phat = M^-1 p
template <class T>
__global__ __launch_bounds__(kVT) void k_bv_p(const int32_t *__restrict__ seg_list, const int *__restrict__ lcount,
                                            const int32_t *__restrict__ seg_sys, const int32_t *__restrict__ seg_off,
                                            const int64_t *__restrict__ row_off, const T *__restrict__ r,
                                            T *__restrict__ p, const T *__restrict__ v, T *__restrict__ ph,
                                            const T *__restrict__ d, const SysState *__restrict__ st,
                                            const int *__restrict__ active) {
    XAB_LISTED_SEGMENT(j);
    const SegRange R = seg_range(j, seg_sys, seg_off, row_off);
    if (!active[R.k]) return;
    const double beta = st[R.k].beta, om = st[R.k].omega;
    XAB_SEG_ROWS(R, i) {
        T pi = (T)((double)r[i] + beta * ((double)p[i] - om * (double)v[i]));
        p[i] = pi;
        ph[i] = d ? (T)((double)pi / (double)d[i]) : pi;
    }
}

// partial <a, b> (and <a, a> when kTwo) of each segment
template <class T, bool kTwo>
__global__ __launch_bounds__(kVT) void k_bv_dot(const int32_t *__restrict__ seg_list, const int *__restrict__ lcount,
                                              const int32_t *__restrict__ seg_sys,
                                              const int32_t *__restrict__ seg_off,
                                              const int64_t *__restrict__ row_off, const T *__restrict__ a,
                                              const T *__restrict__ b, const int *__restrict__ active,
                                              double *__restrict__ part) {
    __shared__ double sh[kVT / xab::kWave];
    XAB_LISTED_SEGMENT(j);
    const SegRange R = seg_range(j, seg_sys, seg_off, row_off);
    if (!active[R.k]) return;
    double ab = 0.0, aa = 0.0;
    XAB_SEG_ROWS(R, i) {
        const double ai = (double)a[i];
        ab += ai * (double)b[i];
        if (kTwo) aa += ai * ai;
    }
    ab = vsum(ab, sh);
    if (kTwo) aa = vsum(aa, sh);
    if (threadIdx.x == 0) {
        part[2 * (int64_t)j] = ab;
        if (kTwo) part[2 * (int64_t)j + 1] = aa;
    }
}

// s = r - alpha v, shat = M^-1 s, partial <s, s>
template <class T>
__global__ __launch_bounds__(kVT) void k_bv_s(const int32_t *__restrict__ seg_list, const int *__restrict__ lcount,
                                            const int32_t *__restrict__ seg_sys, const int32_t *__restrict__ seg_off,
                                            const int64_t *__restrict__ row_off, const T *__restrict__ r,
                                            const T *__restrict__ v, T *__restrict__ s, T *__restrict__ shv,
                                            const T *__restrict__ d, const SysState *__restrict__ st,
                                            const int *__restrict__ active, double *__restrict__ part) {
    __shared__ double sh[kVT / xab::kWave];
    XAB_LISTED_SEGMENT(j);
    const SegRange R = seg_range(j, seg_sys, seg_off, row_off);
    if (!active[R.k]) return;
    const double alpha = st[R.k].alpha;
    double ss = 0.0;
    XAB_SEG_ROWS(R, i) {
        T si = (T)((double)r[i] - alpha * (double)v[i]);
        s[i] = si;
        shv[i] = d ? (T)((double)si / (double)d[i]) : si;
        ss += (double)si * (double)si;
    }
    ss = vsum(ss, sh);
    if (threadIdx.x == 0) part[2 * (int64_t)j] = ss;
}

// x += alpha phat + omega shat, r = s - omega t, partials <r, r> and
// <rhat, r>; a system whose s met the tolerance this iteration takes
// x += alpha phat alone
template <class T>
__global__ __launch_bounds__(kVT) void k_bv_x(const int32_t *__restrict__ seg_list, const int *__restrict__ lcount,
                                            const int32_t *__restrict__ seg_sys, const int32_t *__restrict__ seg_off,
                                            const int64_t *__restrict__ row_off, const T *__restrict__ s,
                                            const T *__restrict__ t, const T *__restrict__ ph,
                                            const T *__restrict__ shv, const T *__restrict__ rh, T *__restrict__ x,
                                            T *__restrict__ r, const SysState *__restrict__ st,
                                            const int *__restrict__ active, const int *__restrict__ early,
                                            double *__restrict__ part) {
    __shared__ double sh[kVT / xab::kWave];
    XAB_LISTED_SEGMENT(j);
    const SegRange R = seg_range(j, seg_sys, seg_off, row_off);
    const double al = st[R.k].alpha;
    if (early[R.k]) {
        XAB_SEG_ROWS(R, i) x[i] = (T)((double)x[i] + al * (double)ph[i]);
        return;
    }
    if (!active[R.k]) return;
    const double om = st[R.k].omega;
    double rr = 0.0, rho = 0.0;
    XAB_SEG_ROWS(R, i) {
        x[i] = (T)((double)x[i] + al * (double)ph[i] + om * (double)shv[i]);
        T ri = (T)((double)s[i] - om * (double)t[i]);
        r[i] = ri;
        rr += (double)ri * (double)ri;
        rho += (double)rh[i] * (double)ri;
    }
    rr = vsum(rr, sh);
    rho = vsum(rho, sh);
    if (threadIdx.x == 0) {
        part[2 * (int64_t)j] = rr;
        part[2 * (int64_t)j + 1] = rho;
    }
}

#undef XAB_SEG_ROWS
#undef XAB_LISTED_SEGMENT

// ---- per-system kernels: one wave per system sums the partials of its
// segments in segment order (a fixed xor tree over the lanes), takes the
// scalar decisions and updates the state and the masks.
__device__ __forceinline__ double seg_total(const double *__restrict__ part, int c, int j0, int j1) {
    double a = 0.0;
    for (int j = j0 + (int)(threadIdx.x % xab::kWave); j < j1; j += xab::kWave) a += part[2 * j + c];
    return xab::wave_sum(a);
}

__device__ __forceinline__ int wave_system() {
    return (int)(blockIdx.x * (kFT / xab::kWave) + threadIdx.x / xab::kWave);
}

// alpha = rho / <rhat, v>; breakdown when <rhat, v> = 0
__global__ __launch_bounds__(kFT) void k_bf_alpha(const int32_t *__restrict__ seg_off, int ns,
                                                const double *__restrict__ part, SysState *__restrict__ st,
                                                int *__restrict__ active, int *__restrict__ n_active) {
    const int k = wave_system();
    if (k >= ns || !active[k]) return;
    const double rv = seg_total(part, 0, seg_off[k], seg_off[k + 1]);
    if (threadIdx.x % xab::kWave) return;
    if (rv == 0.0) {
        st[k].status = 2;
        active[k] = 0;
        atomicSub(n_active, 1);
    } else {
        st[k].alpha = st[k].rho / rv;
    }
}

// ||s|| / ||b|| <= the system's threshold: it stops after x += alpha phat
__global__ __launch_bounds__(kFT) void k_bf_s(const int32_t *__restrict__ seg_off, int ns,
                                            const double *__restrict__ part, SysState *__restrict__ st,
                                            int *__restrict__ active, int *__restrict__ early,
                                            const double *__restrict__ tolv, int *__restrict__ n_active) {
    const int k = wave_system();
    if (k >= ns || !active[k]) return;
    const double ss = seg_total(part, 0, seg_off[k], seg_off[k + 1]);
    if (threadIdx.x % xab::kWave) return;
    const double res = sqrt(ss) / st[k].bnorm;
    if (res <= tolv[k]) {
        SysState q = st[k];
        q.res = res;
        q.iters += 1;
        q.status = 0;
        st[k] = q;
        active[k] = 0;
        early[k] = 1;
        atomicSub(n_active, 1);
    }
}

// omega = <t, s> / <t, t> (0 when t = 0)
__global__ __launch_bounds__(kFT) void k_bf_omega(const int32_t *__restrict__ seg_off, int ns,
                                                const double *__restrict__ part, SysState *__restrict__ st,
                                                const int *__restrict__ active) {
    const int k = wave_system();
    if (k >= ns || !active[k]) return;
    const double ts = seg_total(part, 0, seg_off[k], seg_off[k + 1]);
    const double tt = seg_total(part, 1, seg_off[k], seg_off[k + 1]);
    if (threadIdx.x % xab::kWave) return;
    st[k].omega = tt != 0.0 ? ts / tt : 0.0;
}

// end of an iteration: ||r|| / ||b|| against tol, omega = 0 (breakdown), the
// iteration limit, then rho_next = <rhat, r> (breakdown when 0) and
// beta = (rho_next / rho) (alpha / omega) for the next direction
__global__ __launch_bounds__(kFT) void k_bf_x(const int32_t *__restrict__ seg_off, int ns,
                                            const double *__restrict__ part, SysState *__restrict__ st,
                                            int *__restrict__ active, int *__restrict__ early,
                                            const double *__restrict__ tolv, int64_t maxiter,
                                            int *__restrict__ n_active, int *__restrict__ lcount) {
    if (blockIdx.x == 0 && threadIdx.x < 2) lcount[threadIdx.x] = 0;  // lists of the next iteration
    const int k = wave_system();
    if (k >= ns) return;
    const bool lead = threadIdx.x % xab::kWave == 0;
    if (early[k]) {
        if (lead) early[k] = 0;
        return;
    }
    if (!active[k]) return;
    const double rr = seg_total(part, 0, seg_off[k], seg_off[k + 1]);
    const double rho = seg_total(part, 1, seg_off[k], seg_off[k + 1]);
    if (!lead) return;
    SysState q = st[k];
    q.iters += 1;
    q.res = sqrt(rr) / q.bnorm;
    bool stop = true;
    if (q.res <= tolv[k]) {
        q.status = 0;
    } else if (q.omega == 0.0) {
        q.status = 2;
    } else if (q.iters >= maxiter) {
        // stays "not converged"
    } else if (rho == 0.0) {
        q.status = 2;
    } else {
        stop = false;
        q.beta = (rho / q.rho) * (q.alpha / q.omega);
        q.rho = rho;
    }
    st[k] = q;
    if (stop) {
        active[k] = 0;
        atomicSub(n_active, 1);
    }
}

// true residual per system: res[k] = ||b - A x||_k / ||b||_k (A x given)
template <class T>
__global__ __launch_bounds__(kBiNT) void k_bi_true(const int64_t *__restrict__ row_off, const T *__restrict__ bvec,
                                                 const T *__restrict__ ax, const SysState *__restrict__ st,
                                                 double *__restrict__ out) {
    __shared__ double sh[kBiNT / xab::kWave];
    const int k = blockIdx.x;
    const int64_t r0 = row_off[k], r1 = row_off[k + 1];
    double a = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBiNT) {
        double e = (double)bvec[i] - (double)ax[i];
        a += e * e;
    }
    a = bsum(a, sh);
    if (threadIdx.x == 0) out[k] = sqrt(a) / st[k].bnorm;
}

// system index of every row; columns of system k inside its row range
__global__ void k_sys_of_row(const int64_t *__restrict__ row_off, int32_t nsys, int32_t *__restrict__ sys) {
    const int k = blockIdx.x;
    if (k >= nsys) return;
    for (int64_t i = row_off[k] + threadIdx.x; i < row_off[k + 1]; i += blockDim.x) sys[i] = k;
}

__global__ void k_check_blockdiag(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                  const int64_t *__restrict__ row_off, const int32_t *__restrict__ sys, int64_t n,
                                  int *__restrict__ flag) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int k = sys[r];
    int64_t lo = row_off[k], hi = row_off[k + 1];
    for (int64_t q = rowptr[r]; q < rowptr[r + 1]; ++q)
        if (colind[q] < lo || colind[q] >= hi) {
            atomicOr(flag, 1);
            break;
        }
}

// Jacobi diagonal: 8 lanes per row, each summing the row's diagonal entries
// among its strided share, then a fixed xor tree over the 8 lanes.
template <class T>
__global__ __launch_bounds__(256) void k_diag_b(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                                const T *__restrict__ val, int64_t n, T *__restrict__ d) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 8;
    const int l = threadIdx.x % 8;
    double a = 0.0;
    if (r < n)
        for (int64_t k = rowptr[r] + l; k < rowptr[r + 1]; k += 8)
            if (colind[k] == r) a += (double)val[k];
#pragma unroll
    for (int m = 4; m > 0; m >>= 1) a += __shfl_xor(a, m, 8);
    if (r < n && l == 0) d[r] = a != 0.0 ? (T)a : T(1);
}

__global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0) *p = 0;
}

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }


template <class T>
void launch_batch_spmv(const xab_batch *B, const T *x, T *y, const int *active, hipStream_t st) {
    if (B->sell.cols) {
        const xab_sell &S = B->sell;
        const T *pv;
        if constexpr (sizeof(T) == 8) pv = (const T *)S.val64;
        else pv = (const T *)S.val32;
        const int64_t nwg = (S.nch + kNT / kSellC - 1) / (kNT / kSellC);
        hipLaunchKernelGGL((k_batch_sell<T>), dim3((unsigned)nwg), dim3(kNT), 0, st, S.cptr, S.clen, S.rlen, S.perm,
                           S.cols, pv, x, y, (int32_t)B->n, S.nch, nwg, B->d_sys_of_row, active);
        return;
    }
    hipLaunchKernelGGL((k_batch_spmv<T>), dim3((unsigned)B->P), dim3(kNT), 0, st, B->rowptr, B->colind,
                       (const T *)B->val, x, y, B->nnz, B->P, B->row_lo, B->tile_row, B->carry_row, B->carry_val,
                       B->tail_val, B->tail_row, B->d_sys_of_row, (int32_t)B->n, active);
    hipLaunchKernelGGL((k_batch_fixup<T>), dim3(grid_for(B->P, 256)), dim3(256), 0, st, y, B->P, B->carry_row,
                       B->carry_val, B->tail_val, B->tail_row);
}

template <class T>
int batch_spmv_t(xab_ctx *ctx, const xab_batch *B, const T *x, T *y, const int *active, hipStream_t st) {
    if (B->n == 0) return XAB_OK;
    launch_batch_spmv<T>(B, x, y, active, st);
    XAB_LAUNCH_CHECK(ctx, "k_batch_spmv");
    return XAB_OK;
}

template <class T>
int bicgstab_t(xab_ctx *ctx, const xab_batch *B, const T *bvec, T *x, const xab_krylov_opts *o, xab_krylov_info *hinfo,
               xab_krylov_info *all) {
    const int64_t n = B->n;
    const int ns = B->nsys;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t vb = al(sizeof(T) * (size_t)n);
    size_t off_st = 10 * vb;
    size_t off_act = off_st + al(sizeof(SysState) * ns);
    size_t off_early = off_act + al(sizeof(int) * ns);
    size_t off_cnt = off_early + al(sizeof(int) * ns);
    size_t off_res = off_cnt + 256;
    size_t off_part = off_res + al(sizeof(double) * ns);
    const int64_t nwin = B->sell.cols ? (n + kSellSigma - 1) / kSellSigma : 0;
    size_t off_lseg = off_part + al(sizeof(double) * 2 * (size_t)std::max<int64_t>(B->nseg, 1));
    size_t off_lwin = off_lseg + al(sizeof(int32_t) * (size_t)std::max<int64_t>(B->nseg, 1));
    size_t off_lcnt = off_lwin + al(sizeof(int32_t) * (size_t)std::max<int64_t>(nwin, 1));
    size_t off_tolv = off_lcnt + 256;
    size_t off_redo = off_tolv + al(sizeof(double) * ns);
    size_t total = off_redo + al(sizeof(int) * ns);
    char *w = (char *)xab_dalloc(ctx, total);
    if (!w) return xab_fail(ctx, XAB_E_NOMEM, "BiCGStab workspace");
    T *r = (T *)w, *rh = (T *)(w + vb), *p = (T *)(w + 2 * vb), *v = (T *)(w + 3 * vb), *ph = (T *)(w + 4 * vb);
    T *s = (T *)(w + 5 * vb), *shv = (T *)(w + 6 * vb), *t = (T *)(w + 7 * vb);
    T *ax = (T *)(w + 9 * vb);
    SysState *stt = (SysState *)(w + off_st);
    int *active = (int *)(w + off_act);
    int *early = (int *)(w + off_early);
    int *n_active = (int *)(w + off_cnt);
    double *res = (double *)(w + off_res);
    double *part = (double *)(w + off_part);
    int32_t *seg_list = (int32_t *)(w + off_lseg), *win_list = (int32_t *)(w + off_lwin);
    int *lcount = (int *)(w + off_lcnt);
    double *tolv = (double *)(w + off_tolv);  // each system's threshold (the accuracy policy narrows it)
    int *redo = (int *)(w + off_redo);
    hipStream_t st = ctx->stream;
    hipStream_t gs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&](int code) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (gs) {
            (void)hipStreamSynchronize(gs);
            (void)hipStreamDestroy(gs);
        }
        (void)hipStreamSynchronize(st);
        xab_dfree(ctx, w);
        return code;
    };
    const bool jac = o->precond == XAB_PRECOND_JACOBI;
    const double tol = o->tol;
    const int64_t maxiter = o->maxiter > 0 ? o->maxiter : 10000;
    auto t0 = std::chrono::steady_clock::now();
    int sres;
    if (jac && !B->diag) {
        // computed once per batch and kept with it
        xab_batch *Bm = const_cast<xab_batch *>(B);
        Bm->diag = xab_dalloc(ctx, sizeof(T) * (size_t)(n > 0 ? n : 1));
        if (!Bm->diag) return cleanup(xab_fail(ctx, XAB_E_NOMEM, "Jacobi diagonal"));
        if (n > 0)
            hipLaunchKernelGGL((k_diag_b<T>), dim3(grid_for(n * 8, 256)), dim3(256), 0, st, B->rowptr, B->colind,
                               (const T *)B->val, n, (T *)Bm->diag);
    }
    std::vector<double> htol(ns, tol);
    std::vector<int> hredo(ns, 0), narrowed(ns, 0);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, n_active);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, lcount);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, lcount + 1);
    hipError_t e = hipMemcpyAsync(tolv, htol.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return cleanup(xab_hip_check(ctx, e, "BiCGStab thresholds"));
    if ((sres = batch_spmv_t<T>(ctx, B, x, ax, nullptr, st)) != XAB_OK) return cleanup(sres);
    hipLaunchKernelGGL((k_bi_init<T>), dim3(ns), dim3(kBiNT), 0, st, B->d_row_off, bvec, ax, r, rh, p, v, stt, active,
                       early, tolv, nullptr, n_active);
    e = hipGetLastError();
    if (e != hipSuccess) return cleanup(xab_hip_check(ctx, e, "BiCGStab init"));
    const T *dd = jac ? (const T *)B->diag : nullptr;
    // one iteration over all systems
    const unsigned nseg = (unsigned)B->nseg;
    const unsigned nfw = (unsigned)((ns + kFT / xab::kWave - 1) / (kFT / xab::kWave));
    const unsigned nlist = grid_for(std::max<int64_t>(B->nseg, nwin), 256);
    const unsigned gwin = (unsigned)((nwin * kWinItems + xab::kXcds - 1) / xab::kXcds * xab::kXcds);
    const int32_t *so = B->d_seg_off, *ss = B->d_seg_sys;
    const int64_t *ro = B->d_row_off;
    auto spmv = [&](const T *xin, T *yout, hipStream_t q) {
        if (!nwin) {
            launch_batch_spmv<T>(B, xin, yout, active, q);
            return;
        }
        const xab_sell &S = B->sell;
        const T *pv;
        if constexpr (sizeof(T) == 8) pv = (const T *)S.val64;
        else pv = (const T *)S.val32;
        hipLaunchKernelGGL((k_batch_sell_listed<T>), dim3(gwin), dim3(kNT), 0, q, S.cptr, S.clen, S.rlen, S.perm,
                           S.cols, pv, xin, yout, (int32_t)n, S.nch, win_list, lcount);
    };
    auto enqueue_iter = [&](hipStream_t q) {
        if (nlist)
            hipLaunchKernelGGL(k_bi_lists, dim3(nlist), dim3(256), 0, q, n, B->nseg, nwin, ss, B->d_sys_of_row, active,
                               seg_list, win_list, lcount);
        if (nseg)
            hipLaunchKernelGGL((k_bv_p<T>), dim3(nseg), dim3(kVT), 0, q, seg_list, lcount, ss, so, ro, r, p, v, ph, dd,
                               stt, active);
        spmv(ph, v, q);
        if (nseg)
            hipLaunchKernelGGL((k_bv_dot<T, false>), dim3(nseg), dim3(kVT), 0, q, seg_list, lcount, ss, so, ro, v, rh,
                               active, part);
        hipLaunchKernelGGL(k_bf_alpha, dim3(nfw), dim3(kFT), 0, q, so, ns, part, stt, active, n_active);
        if (nseg)
            hipLaunchKernelGGL((k_bv_s<T>), dim3(nseg), dim3(kVT), 0, q, seg_list, lcount, ss, so, ro, r, v, s, shv, dd,
                               stt, active, part);
        hipLaunchKernelGGL(k_bf_s, dim3(nfw), dim3(kFT), 0, q, so, ns, part, stt, active, early, tolv, n_active);
        spmv(shv, t, q);
        if (nseg)
            hipLaunchKernelGGL((k_bv_dot<T, true>), dim3(nseg), dim3(kVT), 0, q, seg_list, lcount, ss, so, ro, t, s,
                               active, part);
        hipLaunchKernelGGL(k_bf_omega, dim3(nfw), dim3(kFT), 0, q, so, ns, part, stt, active);
        if (nseg)
            hipLaunchKernelGGL((k_bv_x<T>), dim3(nseg), dim3(kVT), 0, q, seg_list, lcount, ss, so, ro, s, t, ph, shv, rh,
                               x, r, stt, active, early, part);
        hipLaunchKernelGGL(k_bf_x, dim3(nfw), dim3(kFT), 0, q, so, ns, part, stt, active, early, tolv, maxiter,
                           n_active, lcount);
    };
    const int every = o->check_every > 0 ? o->check_every : 8;
    hipEvent_t ev = nullptr;
    if (o->graph) {
        // capture on a library stream (the caller's may be the legacy default
        // stream, which cannot be captured), ordered after the caller's work
        e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(gs, ev, 0);
        if (e == hipSuccess) e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int i = 0; i < every; ++i) enqueue_iter(gs);
            e = hipStreamEndCapture(gs, &graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (ev) (void)hipEventDestroy(ev);
            return cleanup(xab_hip_check(ctx, e, "BiCGStab graph"));
        }
    }
    hipStream_t run = o->graph ? gs : st;
    int64_t done_iters = 0;
    std::vector<SysState> hs(ns);
    std::vector<double> hr(ns);
    for (int pass = 0;; ++pass) {
        int h_active = 1;
        while (done_iters < maxiter) {
            if (o->graph) e = hipGraphLaunch(exec, gs);
            else {
                for (int i = 0; i < every; ++i) enqueue_iter(st);
                e = hipGetLastError();
            }
            if (e != hipSuccess) break;
            done_iters += every;
            e = hipMemcpyAsync(&h_active, n_active, sizeof(int), hipMemcpyDeviceToHost, run);
            if (e == hipSuccess) e = hipStreamSynchronize(run);
            if (e != hipSuccess || h_active <= 0) break;
        }
        if (e != hipSuccess) break;
        if (o->graph) {
            e = hipStreamSynchronize(gs);
            if (e != hipSuccess) break;
        }
        // true residuals
        if ((sres = batch_spmv_t<T>(ctx, B, x, ax, nullptr, st)) != XAB_OK) {
            if (ev) (void)hipEventDestroy(ev);
            return cleanup(sres);
        }
        hipLaunchKernelGGL((k_bi_true<T>), dim3(ns), dim3(kBiNT), 0, st, B->d_row_off, bvec, ax, stt, res);
        e = hipMemcpyAsync(hs.data(), stt, sizeof(SysState) * ns, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), res, sizeof(double) * ns, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        // accuracy policy (section 3.3.2): a system whose recurrence met its
        // threshold while its true residual misses tol runs again from its
        // current x with the threshold narrowed tenfold, while iterations
        // remain (at most kMaxNarrow times)
        if (ctx->policy != XAB_ACCURACY || done_iters >= maxiter) break;
        int nredo = 0;
        for (int k = 0; k < ns; ++k) {
            hredo[k] = hs[k].status == 0 && hr[k] > tol && narrowed[k] < kMaxNarrow;
            if (hredo[k]) {
                htol[k] /= 10.0;
                ++narrowed[k];
                ++nredo;
            }
        }
        if (!nredo) break;
        e = hipMemcpyAsync(tolv, htol.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(redo, hredo.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) break;
        // ax = A x is current: the restart starts from the true residual
        hipLaunchKernelGGL((k_bi_init<T>), dim3(ns), dim3(kBiNT), 0, st, B->d_row_off, bvec, ax, r, rh, p, v, stt,
                           active, early, tolv, redo, n_active);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vectors are rewritten by the next pass
        if (e != hipSuccess) break;
        if (o->graph) {
            // the graph's stream runs after the host-side work above
            e = hipEventRecord(ev, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(gs, ev, 0);
            if (e != hipSuccess) break;
        }
    }
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) return cleanup(xab_hip_check(ctx, e, "BiCGStab iterations"));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int agg = XAB_OK;
    int64_t maxit = 0;
    double worst = 0.0;
    for (int k = 0; k < ns; ++k) {
        int sk = hs[k].status == 0 ? XAB_OK : (hs[k].status == 2 ? XAB_BREAKDOWN : XAB_NOT_CONVERGED);
        // accuracy policy: a convergence the true residual does not confirm
        // (narrowing cap or iteration limit reached) is not a convergence
        if (sk == XAB_OK && ctx->policy == XAB_ACCURACY && !(hr[k] <= tol)) sk = XAB_NOT_CONVERGED;
        if (sk == XAB_BREAKDOWN) agg = XAB_BREAKDOWN;
        else if (sk == XAB_NOT_CONVERGED && agg == XAB_OK) agg = XAB_NOT_CONVERGED;
        maxit = std::max<int64_t>(maxit, hs[k].iters);
        worst = std::max(worst, hr[k]);
        if (hinfo) {
            hinfo[k] = xab_krylov_info{};
            hinfo[k].iters = hs[k].iters;
            hinfo[k].true_relres = hr[k];
            hinfo[k].seconds = secs;
            hinfo[k].status = sk;
            hinfo[k].faults = narrowed[k];
        }
    }
    if (all) {
        *all = xab_krylov_info{};
        all->iters = maxit;
        all->restarts = done_iters;
        all->true_relres = worst;
        all->seconds = secs;
        all->status = agg;
    }
    return cleanup(agg);
}

}  // namespace

extern "C" {

int xab_batch_csr(xab_ctx *ctx, int32_t nsys, const int64_t *h_row_off, const int64_t *h_nnz_off,
                  const int32_t *d_rowptr, const int32_t *d_colind, const void *d_val, xab_dtype vt, uint32_t flags,
                  xab_batch **out) {
    if (!ctx || !out || !h_row_off || !h_nnz_off) return XAB_E_NULL;
    *out = nullptr;
    if (nsys < 1) return xab_fail(ctx, XAB_E_SHAPE, "nsys = %d", nsys);
    if (vt != XAB_F64 && vt != XAB_F32) return xab_fail(ctx, XAB_E_DTYPE, "value type");
    if (h_row_off[0] != 0 || h_nnz_off[0] != 0) return xab_fail(ctx, XAB_E_SHAPE, "offsets must start at 0");
    for (int k = 0; k < nsys; ++k)
        if (h_row_off[k + 1] < h_row_off[k] || h_nnz_off[k + 1] < h_nnz_off[k])
            return xab_fail(ctx, XAB_E_SHAPE, "offsets must be monotone");
    const int64_t n = h_row_off[nsys], nnz = h_nnz_off[nsys];
    if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31)) return xab_fail(ctx, XAB_E_SHAPE, "batch too large");
    xab_matrix *A = nullptr;
    int s = xab_matrix_csr(ctx, (int32_t)n, (int32_t)n, nnz, d_rowptr, d_colind, d_val, vt, flags & XAB_TRUST_INPUT, &A);
    if (s != XAB_OK) return s;
    xab_batch *B = new xab_batch();
    B->ctx = ctx;
    B->nsys = nsys;
    B->n = n;
    B->nnz = nnz;
    B->row_off.assign(h_row_off, h_row_off + nsys + 1);
    B->nnz_off.assign(h_nnz_off, h_nnz_off + nsys + 1);
    B->rowptr = d_rowptr;
    B->colind = d_colind;
    B->val = d_val;
    B->vt = vt;
    xab_matrix_destroy(A);
    const int64_t T = (int64_t)kNT * kBatchJ;
    B->P = std::max<int64_t>(1, (nnz + T - 1) / T);
    B->row_lo = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (B->P + 1));
    B->tile_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (B->P + 1));
    B->carry_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * B->P);
    B->tail_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * B->P);
    B->carry_val = (double *)xab_dalloc(ctx, sizeof(double) * B->P);
    B->tail_val = (double *)xab_dalloc(ctx, sizeof(double) * B->P);
    B->d_sys_of_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (n > 0 ? n : 1));
    B->d_row_off = (int64_t *)xab_dalloc(ctx, sizeof(int64_t) * (nsys + 1));
    // segments of kSegRows rows for the BiCGStab row kernels
    std::vector<int32_t> seg_off(nsys + 1), seg_sys;
    for (int k = 0; k < nsys; ++k) {
        seg_off[k] = (int32_t)seg_sys.size();
        seg_sys.resize(seg_sys.size() + (size_t)((h_row_off[k + 1] - h_row_off[k] + kSegRows - 1) / kSegRows), k);
    }
    seg_off[nsys] = (int32_t)seg_sys.size();
    B->nseg = (int64_t)seg_sys.size();
    B->d_seg_off = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (nsys + 1));
    B->d_seg_sys = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * std::max<size_t>(seg_sys.size(), 1));
    if (!B->row_lo || !B->tile_row || !B->carry_row || !B->tail_row || !B->carry_val || !B->tail_val ||
        !B->d_sys_of_row || !B->d_row_off || !B->d_seg_off || !B->d_seg_sys) {
        xab_batch_destroy(B);
        return xab_fail(ctx, XAB_E_NOMEM, "batch plan");
    }
    hipStream_t st = ctx->stream;
    hipError_t e = hipMemcpyAsync(B->d_row_off, h_row_off, sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->d_seg_off, seg_off.data(), sizeof(int32_t) * (nsys + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !seg_sys.empty())
        e = hipMemcpyAsync(B->d_seg_sys, seg_sys.data(), sizeof(int32_t) * seg_sys.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        xab_launch_split_bss(st, d_rowptr, (int32_t)n, T, B->P, B->row_lo, B->tile_row, B->carry_row);
        hipLaunchKernelGGL(k_sys_of_row, dim3(nsys), dim3(256), 0, st, B->d_row_off, nsys, B->d_sys_of_row);
        if (!(flags & XAB_TRUST_INPUT) && n > 0) {
            hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, ctx->d_flag);
            hipLaunchKernelGGL(k_check_blockdiag, dim3(grid_for(n, 256)), dim3(256), 0, st, d_rowptr, d_colind,
                               B->d_row_off, B->d_sys_of_row, n, ctx->d_flag);
        }
        e = hipGetLastError();
    }
    int hflag = 0;
    if (e == hipSuccess && !(flags & XAB_TRUST_INPUT))
        e = hipMemcpyAsync(&hflag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        xab_batch_destroy(B);
        return xab_hip_check(ctx, e, "batch setup");
    }
    if (hflag) {
        xab_batch_destroy(B);
        return xab_fail(ctx, XAB_E_STRUCT, "a system has columns outside its own rows");
    }
    // the sliced ELLPACK copy, unless asked for the tiles alone; outside its
    // limits, or without the memory for it, the tiles serve
    if (!(flags & XAB_BATCH_TILES) && n > 0) {
        s = xab_sell_build(ctx, d_rowptr, d_colind, vt == XAB_F64 ? (const double *)d_val : nullptr,
                           vt == XAB_F32 ? (const float *)d_val : nullptr, vt == XAB_F64, vt == XAB_F32, (int32_t)n,
                           nnz, kSellSigma, &B->sell);
        if (s != XAB_OK && s != XAB_E_UNSUPPORTED && s != XAB_E_NOMEM) {
            xab_batch_destroy(B);
            return s;
        }
    }
    *out = B;
    return XAB_OK;
}

void xab_batch_destroy(xab_batch *B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->ctx->stream);
    xab_dfree(B->ctx, B->row_lo);
    xab_dfree(B->ctx, B->tile_row);
    xab_dfree(B->ctx, B->carry_row);
    xab_dfree(B->ctx, B->tail_row);
    xab_dfree(B->ctx, B->carry_val);
    xab_dfree(B->ctx, B->tail_val);
    xab_dfree(B->ctx, B->diag);
    xab_dfree(B->ctx, B->d_sys_of_row);
    xab_dfree(B->ctx, B->d_row_off);
    xab_dfree(B->ctx, B->d_seg_off);
    xab_dfree(B->ctx, B->d_seg_sys);
    xab_sell_free(B->ctx, &B->sell);
    delete B;
}

int xab_batch_layout(const xab_batch *B) {
    if (!B) return -1;
    return B->sell.cols ? 1 : 0;
}

int xab_batch_spmv(xab_ctx *ctx, const xab_batch *B, const void *d_x, void *d_y) {
    if (!ctx || !B || !d_x || !d_y) return XAB_E_NULL;
    if (d_x == d_y) return xab_fail(ctx, XAB_E_ALIAS, "x and y alias");
    if (B->vt == XAB_F64) return batch_spmv_t<double>(ctx, B, (const double *)d_x, (double *)d_y, nullptr, ctx->stream);
    return batch_spmv_t<float>(ctx, B, (const float *)d_x, (float *)d_y, nullptr, ctx->stream);
}

int xab_bicgstab(xab_ctx *ctx, const xab_batch *B, const void *d_b, void *d_x, const xab_krylov_opts *opts,
                 xab_krylov_info *h_info, xab_krylov_info *all) {
    if (!ctx || !B || !d_b || !d_x || !opts) return XAB_E_NULL;
    if (d_b == d_x) return xab_fail(ctx, XAB_E_ALIAS, "b and x alias");
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    if (B->vt == XAB_F64)
        return bicgstab_t<double>(ctx, B, (const double *)d_b, (double *)d_x, opts, h_info, all);
    return bicgstab_t<float>(ctx, B, (const float *)d_b, (float *)d_x, opts, h_info, all);
}

}  // extern "C"
