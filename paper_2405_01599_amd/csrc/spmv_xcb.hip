// Column-blocked segmented-scan SpMV (one column block per XCD).
#include "segchunk.h"
#include "spmv_launch.h"

namespace xab {
namespace {

constexpr int kNT = 256;  // threads per workgroup

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------------ XCB
// Column-blocked segmented scan.  The columns are cut into kXcds blocks;
// block k's entries form their own CSR over the rows that have entries in
// the block (its compressed rows, built at plan time), and bit 31 of a
// column index flags the first entry of each compressed row: the flag
// array of the segmented-scan format folded into the columns, so a tile
// finds its row starts without reading any row pointer.  Workgroup ids are
// dealt round-robin to the XCDs; giving block k every id with
// id % kXcds == k keeps its gathers on one XCD, whose private L2 then holds
// that block's slice of x.
// Tile t of block k covers entries [tT, tT + T) (a full tile is stored in
// lane-interleaved 16-byte groups, see load_tile_grouped).  Its first entry lies in
// compressed row row0[t], so entry e lies in row
// row0[t] - head(tT) + (heads in [tT, e]).  A block writes one partial per
// compressed row into its slice of Y; the combine kernel adds, for every
// row, the partials of the blocks its mask names, in block order.
struct XcbArgs {
    const int32_t *colind[kXcds];  // flagged
    const void *val[kXcds];
    const int32_t *row0[kXcds];    // per tile: compressed row holding its first entry
    const int32_t *carry_row[kXcds];
    void *carry_val[kXcds];
    void *tail_val[kXcds];
    int32_t *tail_row[kXcds];
    void *Y[kXcds];                // compressed partials of each block
    int64_t nnz[kXcds];
    int64_t P[kXcds];
};

// A full tile stores each lane's J entries in groups of G = min(J, 16 /
// element size) consecutive entries, group c of lane t at (c 256 + t) G:
// each 16-byte (or narrower) load of the workgroup reads one contiguous run
template <class T, int J>
__device__ __forceinline__ void load_tile_grouped(const T *__restrict__ p, int tid, T (&out)[J]) {
    constexpr int G = J < 16 / (int)sizeof(T) ? J : 16 / (int)sizeof(T);
    if constexpr (G == 1) {
#pragma unroll
        for (int q = 0; q < J; ++q) out[q] = __builtin_nontemporal_load(p + q * kNT + tid);
    } else {
        typedef T V __attribute__((ext_vector_type(G)));
        const V *vp = reinterpret_cast<const V *>(p);
#pragma unroll
        for (int c = 0; c < J / G; ++c) {
            const V w = __builtin_nontemporal_load(vp + c * kNT + tid);
#pragma unroll
            for (int i = 0; i < G; ++i) out[c * G + i] = w[i];
        }
    }
}

template <class VT, class XT, class AT, int J>
__global__ __launch_bounds__(kNT) void k_spmv_xcb(XcbArgs a, const XT *__restrict__ x) {
    constexpr int T = kNT * J;
    constexpr int NW = kNT / kWave;
    __shared__ CSeg<AT> wave_tot[NW];
    // partials of the rows that start in the tile: the first YS of them
    // (all, on matrices whose compressed rows average two entries or more)
    // are staged, any further ones written directly
    constexpr int YS = T < 4096 ? T : 4096;
    __shared__ AT ys[YS];
    const int k = blockIdx.x % kXcds;
    const int64_t t = blockIdx.x / kXcds;
    const int64_t nnz = a.nnz[k];
    if (t >= a.P[k] || nnz == 0) return;
    const int32_t *__restrict__ ci = a.colind[k];
    const VT *__restrict__ va = (const VT *)a.val[k];
    AT *__restrict__ Y = (AT *)a.Y[k];
    const int64_t A0 = t * T, c1 = A0 + T < nnz ? A0 + T : nnz;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;

    int32_t cr[J];
    VT v[J];
    const int64_t base = A0 + (int64_t)tid * J;
    if (A0 + T <= nnz) {
        load_tile_grouped<int32_t, J>(ci + A0, tid, cr);
        load_tile_grouped<VT, J>(va + A0, tid, v);
    } else {
#pragma unroll
        for (int q = 0; q < J; ++q) {
            const bool live = base + q < c1;
            cr[q] = live ? __builtin_nontemporal_load(ci + base + q) : kDeadCol;
            v[q] = live ? __builtin_nontemporal_load(va + base + q) : VT(0);
        }
    }
    const int h0 = ci[A0] < 0;                        // does a row start at the tile's first entry
    const int hnext = c1 < nnz ? (ci[c1] < 0) : 1;     // does the last row end inside the tile
    const int32_t r0 = a.row0[k][t] - h0;
    XT xv[J];
    int hd[J];
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int32_t c = cr[q];
        hd[q] = (c < 0) & (c != kDeadCol);
        xv[q] = c != kDeadCol ? x[c & 0x7fffffff] : XT(0);
    }
    AT p[J];
#pragma unroll
    for (int q = 0; q < J; ++q) p[q] = (AT)v[q] * (AT)xv[q];

    CSeg<AT> s{0, AT(0)};
#pragma unroll
    for (int q = 0; q < J; ++q) {
        s.v = hd[q] ? p[q] : s.v + p[q];
        s.c += hd[q];
    }
    s = wave_scan_dpp(s, CSegStep{});
    if (lane == kWave - 1) wave_tot[wid] = s;
    __syncthreads();
    CSeg<AT> pre{0, AT(0)}, total{0, AT(0)};
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const CSeg<AT> tw = wave_tot[w];
        if (w < wid) pre = cseg_combine(pre, tw);
        total = cseg_combine(total, tw);
    }
    const CSeg<AT> ex{shfl_up(s.c, 1), shfl_up(s.v, 1)};
    const CSeg<AT> in = lane == 0 ? pre : cseg_combine(pre, ex);

    // pass 2: a head closes the open segment: a row of this tile (heads
    // before it > 0), staged in LDS so that the tile's rows leave in one
    // contiguous run, or the carried-in row's part in this tile
    AT acc = in.v;
    int cnt = in.c;
#pragma unroll
    for (int q = 0; q < J; ++q) {
        if (hd[q]) {
            if (cnt > 0) {
                if (cnt <= YS) ys[cnt - 1] = acc;
                else Y[r0 + cnt] = acc;
            } else if (!h0) {
                ((AT *)a.carry_val[k])[t] = acc;
            }
            acc = p[q];
            ++cnt;
        } else {
            acc += p[q];
        }
    }
    // rows r0 + 1 .. r0 + total.c start in the tile; the last one is
    // complete here only when the next tile starts a row
    const int nrows = total.c > 0 ? total.c - 1 + hnext : 0;
    if (tid == 0) {
        int32_t tr = -1;
        if (total.c == 0) {
            // no row starts in the tile: all of it belongs to the carried row
            ((AT *)a.carry_val[k])[t] = total.v;
        } else if (hnext) {
            if (total.c <= YS) ys[total.c - 1] = total.v;
            else Y[r0 + total.c] = total.v;
        } else {
            tr = r0 + total.c;
            ((AT *)a.tail_val[k])[t] = total.v;
        }
        a.tail_row[k][t] = tr;
    }
    __syncthreads();
    const int staged = nrows < YS ? nrows : YS;
    for (int i = tid; i < staged; i += kNT) Y[r0 + 1 + i] = ys[i];
}

// rows cut by a tile end: their start partial plus the carries of the
// following tiles, in ascending tile order
template <class AT>
__global__ void k_xcb_fixup(XcbArgs a, int64_t pmax) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = (int)(g / pmax);
    const int64_t t = g % pmax;
    if (k >= kXcds || t >= a.P[k] || a.nnz[k] == 0) return;
    const int32_t r = a.tail_row[k][t];
    if (r < 0) return;
    const AT *cv = (const AT *)a.carry_val[k];
    AT acc = ((const AT *)a.tail_val[k])[t];
    for (int64_t u = t + 1; u < a.P[k] && a.carry_row[k][u] == r; ++u) acc += cv[u];
    ((AT *)a.Y[k])[r] = acc;
}

// y_i = sum over the blocks row i has entries in (mask bit k), in block
// order.  Workgroup g covers rows [256g, 256g + 256); the compressed index
// of row i in block k is gbase[k][g] plus the rows of the group before i
// with bit k, counted with wave ballots.
// A sliced plan runs one such product per column slice: the first starts
// the accumulation-type sum ysum (mode 1), the middle ones add to it (2),
// the last adds and writes y (3); an unsliced plan writes y directly (0).
template <class YT, class AT>
__global__ __launch_bounds__(kNT) void k_xcb_combine(XcbArgs a, const uint8_t *__restrict__ mask,
                                                     const int32_t *__restrict__ gbase, int64_t G, int64_t n,
                                                     YT *__restrict__ y, AT *__restrict__ ysum, int mode) {
    constexpr int NW = kNT / kWave;
    __shared__ int wcnt[kXcds][NW];
    const int64_t g = blockIdx.x;
    const int64_t i = g * kNT + threadIdx.x;
    const uint32_t m = i < n ? mask[i] : 0u;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const unsigned long long below = (1ull << lane) - 1ull;
    int pre[kXcds];
#pragma unroll
    for (int k = 0; k < kXcds; ++k) {
        const unsigned long long bal = __ballot((m >> k) & 1u);
        pre[k] = __popcll(bal & below);
        if (lane == 0) wcnt[k][w] = __popcll(bal);
    }
    __syncthreads();
    if (i >= n) return;
    // every block's partial is fetched under its mask bit before any is
    // added, so the up to 8 loads are in flight together; the sum still
    // runs in block order over the set bits
    AT v[kXcds];
#pragma unroll
    for (int k = 0; k < kXcds; ++k) {
        int64_t off = (int64_t)gbase[(int64_t)k * (G + 1) + g] + pre[k];
        for (int q = 0; q < w; ++q) off += wcnt[k][q];
        v[k] = ((m >> k) & 1u) ? ((const AT *)a.Y[k])[off] : AT(0);
    }
    AT acc = mode >= 2 ? ysum[i] : AT(0);
#pragma unroll
    for (int k = 0; k < kXcds; ++k) acc = ((m >> k) & 1u) ? acc + v[k] : acc;
    if (mode == 1 || mode == 2) ysum[i] = acc;
    else y[i] = (YT)acc;
}

}  // namespace

// The arrays of one walk of the blocked copy: the FP64 one, or the FP32
// values' own when the plan made one
struct XcbWalk {
    const int32_t *colind;
    const int64_t *P, *toff;
    int32_t *tile_row, *carry_row, *tail_row;
    void *carry_val, *tail_val;
};

template <class VT, class XT, class YT, class AT, int J>
static int launch_xcb_j(xab_ctx *ctx, const xab_plan *pl, const XcbWalk &wk, const XT *x, YT *y, AT *ysum,
                        int mode) {
    const xab_matrix *A = pl->A;
    constexpr int KB = xab_plan::kXcb;
    static_assert(KB == kXcds, "one column block per XCD");
    const int64_t n = A->n;
    if (n == 0) return XAB_OK;
    XcbArgs a;
    int64_t pmax = 1;
    AT *Y = (AT *)pl->xcb_Y;
    for (int k = 0; k < KB; ++k) {
        const int64_t b = pl->xcb_base[k], o = wk.toff[k];
        a.colind[k] = wk.colind + b;
        if constexpr (sizeof(VT) == 8) a.val[k] = pl->xcb_val64 + b;
        else a.val[k] = pl->xcb_val32 + b;
        a.row0[k] = wk.tile_row + o;
        a.carry_row[k] = wk.carry_row + o;
        a.tail_row[k] = wk.tail_row + o;
        a.carry_val[k] = (AT *)wk.carry_val + o;
        a.tail_val[k] = (AT *)wk.tail_val + o;
        a.Y[k] = Y + pl->xcb_ybase[k];
        a.nnz[k] = pl->xcb_base[k + 1] - b;
        a.P[k] = wk.P[k];
        pmax = std::max(pmax, wk.P[k]);
    }
    hipLaunchKernelGGL((k_spmv_xcb<VT, XT, AT, J>), dim3((unsigned)(KB * pmax)), dim3(kNT), 0, ctx->stream, a, x);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_xcb");
    hipLaunchKernelGGL((k_xcb_fixup<AT>), dim3(grid_for(KB * pmax, 256)), dim3(256), 0, ctx->stream, a, pmax);
    XAB_LAUNCH_CHECK(ctx, "k_xcb_fixup");
    hipLaunchKernelGGL((k_xcb_combine<YT, AT>), dim3((unsigned)pl->xcb_G), dim3(kNT), 0, ctx->stream, a,
                       pl->xcb_mask, pl->xcb_gbase, pl->xcb_G, n, y, ysum, mode);
    XAB_LAUNCH_CHECK(ctx, "k_xcb_combine");
    return XAB_OK;
}

// One product of one XCB plan (the whole matrix, or one column slice).
template <class VT, class XT, class YT, class AT>
static int launch_xcb_plan(xab_ctx *ctx, const xab_plan *pl, const XT *x, YT *y, AT *ysum, int mode) {
    if ((sizeof(VT) == 8 && !pl->xcb_val64) || (sizeof(VT) == 4 && !pl->xcb_val32))
        return xab_fail(ctx, XAB_E_DTYPE, "column-blocked plan holds no values of this precision");
    const bool own32 = sizeof(VT) == 4 && pl->xcb_j32 > 0;
    const XcbWalk wk = own32 ? XcbWalk{pl->xcb_colind32, pl->xcb_P32, pl->xcb_toff32, pl->xcb_tile_row32,
                                       pl->xcb_carry_row32, pl->xcb_tail_row32, pl->xcb_carry_val32,
                                       pl->xcb_tail_val32}
                             : XcbWalk{pl->xcb_colind, pl->xcb_P, pl->xcb_toff, pl->xcb_tile_row, pl->xcb_carry_row,
                                       pl->xcb_tail_row, pl->xcb_carry_val, pl->xcb_tail_val};
    switch (own32 ? pl->xcb_j32 : pl->params.j_per_lane) {
        case 1: return launch_xcb_j<VT, XT, YT, AT, 1>(ctx, pl, wk, x, y, ysum, mode);
        case 2: return launch_xcb_j<VT, XT, YT, AT, 2>(ctx, pl, wk, x, y, ysum, mode);
        case 4: return launch_xcb_j<VT, XT, YT, AT, 4>(ctx, pl, wk, x, y, ysum, mode);
        case 8: return launch_xcb_j<VT, XT, YT, AT, 8>(ctx, pl, wk, x, y, ysum, mode);
        case 16: return launch_xcb_j<VT, XT, YT, AT, 16>(ctx, pl, wk, x, y, ysum, mode);
        case 32: return launch_xcb_j<VT, XT, YT, AT, 32>(ctx, pl, wk, x, y, ysum, mode);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane %d", pl->params.j_per_lane);
    }
}

template <class VT, class XT, class YT, class AT>
int launch_xcb(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    (void)val;  // the plan holds its own column-blocked copy of the values
    if (pl->xcb_sub.empty()) return launch_xcb_plan<VT, XT, YT, AT>(ctx, pl, x, y, nullptr, 0);
    // column slices one after another, summed in slice order
    AT *ysum = (AT *)pl->xcb_ysum;
    const size_t S = pl->xcb_sub.size();
    for (size_t s = 0; s < S; ++s) {
        const int mode = s == 0 ? 1 : (s + 1 < S ? 2 : 3);
        const int st = launch_xcb_plan<VT, XT, YT, AT>(ctx, pl->xcb_sub[s], x, y, ysum, mode);
        if (st != XAB_OK) return st;
    }
    return XAB_OK;
}

XAB_INSTANTIATE_LAUNCHER(launch_xcb)

}  // namespace xab
