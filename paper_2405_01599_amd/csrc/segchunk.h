// Branchless segmented reduction of one chunk of the CRS entry stream.
//
// A workgroup of NT threads covers NT*J consecutive entries [A, A + NT*J)
// of the matrix; lane t owns the J entries starting at A + t*J.  Only the
// entries in [c0, c1) are live.  The products val * x[col] are summed per
// row with the segmented-scan idea the paper's third SpMV uses: a "head"
// marks each entry that starts a row, and every lane runs the same
// branch-free select chain over its J products (new segment at a head,
// accumulate otherwise).  Lane results are joined by a segmented scan
// across the wave (shuffles) and across waves (LDS), so no lane ever
// waits on a row boundary and rows of any length cost the same per entry.
//
// Heads are given as head_row[q - A] = row starting at entry q, or -1
// (written by mark_rows from rowptr; empty rows never start a segment).
//
// The caller seeds the scan with the row left open by the previous chunk
// (K2, symmetric tiles) or with nothing (segmented-scan tiles), and gets
// back the state after the chunk: the row still open and its partial sum.
// Rows that end inside the chunk are handed to sink.row_done(row, sum) by
// the lane that sees the next head.  The partial that precedes the first
// head of the chunk (the tail of a row started before A, when no seed
// carries it) is returned as `lead`.
#pragma once
#include "internal.h"

namespace xab {

template <class T, int J>
__device__ __forceinline__ void load_run_full(const T *__restrict__ p, int64_t base, T (&out)[J]) {
    constexpr int kPer16 = 16 / (int)sizeof(T);
    if constexpr (J % kPer16 == 0) {
        typedef T V __attribute__((ext_vector_type(kPer16)));
        const V *vp = reinterpret_cast<const V *>(p + base);
#pragma unroll
        for (int c = 0; c < J / kPer16; ++c) {
            V v = __builtin_nontemporal_load(vp + c);
#pragma unroll
            for (int i = 0; i < kPer16; ++i) out[c * kPer16 + i] = v[i];
        }
    } else {
#pragma unroll
        for (int k = 0; k < J; ++k) out[k] = __builtin_nontemporal_load(p + base + k);
    }
}

// Row starts of a chunk [A, Aend).  Candidate rows are taken 256 at a time
// from `rlo`; a candidate starts in the chunk when r < rend and (all or
// rowptr[r] < Aend); rowptr is monotone, so these form a prefix and a
// block-wide count gives the next first row.  Non-empty rows write
// head_row[rowptr[r] - A] = r, empty rows go to sink.empty_row.  The first
// candidate's two row pointers (q0, q1) are loaded by the caller
// (first_row) ahead of other work to overlap their latency; head_row must
// hold -1 everywhere and that clearing must be complete (a barrier) first.
// Returns one past the last row that starts in the chunk.
struct RowProbe {
    int32_t r, q0, q1;
};

template <int NT>
__device__ __forceinline__ RowProbe first_row(const int32_t *__restrict__ rowptr, int32_t rlo, int32_t rend) {
    RowProbe p;
    p.r = rlo + (int32_t)threadIdx.x;
    p.q0 = p.r < rend ? rowptr[p.r] : 0;
    p.q1 = p.r < rend ? rowptr[p.r + 1] : 0;
    return p;
}

template <int NT, class Sink>
__device__ __forceinline__ int32_t mark_rows(const int32_t *__restrict__ rowptr, RowProbe p, int32_t rlo,
                                             int32_t rend, int64_t A, int64_t Aend, bool all, int32_t *head_row,
                                             Sink &sink) {
    int32_t rhi = rlo;
    for (;;) {
        const bool pred = p.r < rend && (all || p.q0 < Aend);
        if (pred) {
            if (p.q1 > p.q0) head_row[p.q0 - A] = p.r;
            else sink.empty_row(p.r);
        }
        const int cnt = __syncthreads_count(pred);
        rhi += cnt;
        if (cnt < NT) break;
        p.r += NT;
        p.q0 = p.r < rend ? rowptr[p.r] : 0;
        p.q1 = p.r < rend ? rowptr[p.r + 1] : 0;
    }
    return rhi;
}

template <int NT, int J>
__device__ __forceinline__ void clear_heads(int32_t *head_row) {
#pragma unroll
    for (int k = 0; k < J; ++k) head_row[k * NT + threadIdx.x] = -1;
}

template <class AT>
struct ChunkResult {
    Seg<AT> state;  // block-uniform: row open after the chunk (f = 1) and its partial
    AT lead;        // sum before the first head when no seed row was open
    int has_lead;   // this lane produced `lead`
};

// The lane's J entries of a chunk: values, columns and gathered x values
// (dead slots hold v = 0, col = -1, xv = 0).  Loading is split in two so
// kernels can overlap the latencies: run_load issues the value / column
// loads, run_gather the x gathers (it waits only for the columns).
template <int J, class VT, class XT>
struct Run {
    VT v[J];
    int32_t col[J];
    XT xv[J];
};

template <int NT, int J, class VT, class XT>
__device__ __forceinline__ void run_load(Run<J, VT, XT> &R, int64_t A, int64_t c0, int64_t c1,
                                         const int32_t *__restrict__ colind, const VT *__restrict__ val) {
    const int64_t base = A + (int64_t)threadIdx.x * J;
    if (base >= c0 && base + J <= c1) {
        load_run_full<int32_t, J>(colind, base, R.col);
        load_run_full<VT, J>(val, base, R.v);
    } else {
#pragma unroll
        for (int k = 0; k < J; ++k) {
            int64_t q = base + k;
            bool live = q >= c0 && q < c1;
            R.col[k] = live ? __builtin_nontemporal_load(colind + q) : -1;
            R.v[k] = live ? __builtin_nontemporal_load(val + q) : VT(0);
        }
    }
}

template <int J, class VT, class XT>
__device__ __forceinline__ void run_gather(Run<J, VT, XT> &R, const XT *__restrict__ x) {
#pragma unroll
    for (int k = 0; k < J; ++k) R.xv[k] = R.col[k] >= 0 ? x[R.col[k]] : XT(0);
}

template <int NT, int J, class VT, class XT, class AT, class Sink>
__device__ __forceinline__ ChunkResult<AT> seg_chunk(const Run<J, VT, XT> &R, const int32_t *head_row,
                                                     Seg<AT> seed, Seg<AT> *wave_tot, Sink &sink) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    AT p[J];
    int32_t hr[J];
#pragma unroll
    for (int k = 0; k < J; ++k) p[k] = (AT)R.v[k] * (AT)R.xv[k];
#pragma unroll
    for (int k = 0; k < J; ++k) hr[k] = head_row[tid * J + k];

    // lane aggregate: (any head, sum since the last head, row of the last head)
    Seg<AT> s{0, AT(0), -1};
#pragma unroll
    for (int k = 0; k < J; ++k) {
        int h = hr[k] >= 0;
        s.v = h ? p[k] : s.v + p[k];
        s.r = h ? hr[k] : s.r;
        s.f |= h;
    }
    Seg<AT> incl = wave_seg_scan<AT>(s, lane);
    if (lane == kWave - 1) wave_tot[wid] = incl;
    __syncthreads();
    Seg<AT> pre = seed, total = seed;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        Seg<AT> t = wave_tot[w];
        if (w < wid) pre = seg_combine(pre, t);
        total = seg_combine(total, t);
    }
    Seg<AT> ex;
    ex.f = shfl_up(incl.f, 1);
    ex.v = shfl_up(incl.v, 1);
    ex.r = shfl_up(incl.r, 1);
    Seg<AT> carry = lane == 0 ? pre : seg_combine(pre, ex);

    // pass 2: walk the lane's entries again with the carried-in state
    ChunkResult<AT> res;
    res.state = total;
    res.lead = AT(0);
    res.has_lead = 0;
    AT acc = carry.v;
    int32_t row = carry.r;
    int open = carry.f;
#pragma unroll
    for (int k = 0; k < J; ++k) {
        if (hr[k] >= 0) {
            if (open) sink.row_done(row, acc);
            else {
                res.lead = acc;
                res.has_lead = 1;
            }
            acc = p[k];
            row = hr[k];
            open = 1;
        } else {
            acc += p[k];
        }
        sink.entry(row, R.col[k], R.v[k]);
    }
    return res;
}

// ------------------------------------------------------------------ flagged entry streams
// Plan-owned copies of the column indices can carry the head flags in bit
// 31 (the first entry of every non-empty row).  Kernels over such a stream
// count heads to find rows instead of reading row pointers.

// scan element over flagged entries: heads seen, sum since the last head
template <class AT>
struct CSeg {
    int c;
    AT v;
};
template <class AT>
__device__ __forceinline__ CSeg<AT> cseg_combine(const CSeg<AT> &a, const CSeg<AT> &b) {
    return CSeg<AT>{a.c + b.c, b.c ? b.v : a.v + b.v};
}

struct CSegStep {
    template <int CTRL, int RM, class AT>
    __device__ __forceinline__ CSeg<AT> apply(const CSeg<AT> &s) const {
        const CSeg<AT> u{dpp_move<CTRL, RM>(s.c), dpp_move<CTRL, RM>(s.v)};
        return cseg_combine(u, s);
    }
};

// a live flagged column is never -1: flagged values are INT_MIN + col with
// col < 2^31 - 1, so -1 can mark the dead slots outside the live range
constexpr int32_t kDeadCol = -1;

__device__ __forceinline__ int is_head(int32_t c) { return (c < 0) & (c != kDeadCol); }
__device__ __forceinline__ int32_t col_of(int32_t c) { return c == kDeadCol ? kDeadCol : (c & 0x7fffffff); }



template <int J, class VT, class XT>
__device__ __forceinline__ void run_gather_flagged(Run<J, VT, XT> &R, const XT *__restrict__ x) {
#pragma unroll
    for (int k = 0; k < J; ++k) R.xv[k] = R.col[k] != kDeadCol ? x[R.col[k] & 0x7fffffff] : XT(0);
}

// One chunk of a flagged stream whose tile starts at a row start.  `seed`
// holds the heads seen in the tile before the chunk and the open row's
// partial.  Rows are numbered 0, 1, ... from the tile's first head: at
// every head after the first, the lane hands the finished row to
// sink.row_done(row, sum), and every entry goes to sink.entry(row, col,
// val) (dead slots with col = kDeadCol).  Returns the block-uniform state
// after the chunk.  Contains two barriers; the second makes wave_tot free
// for the next chunk.
template <int NT, int J, class VT, class XT, class AT, class Sink>
__device__ __forceinline__ CSeg<AT> flag_chunk(const Run<J, VT, XT> &R, CSeg<AT> seed, CSeg<AT> *wave_tot,
                                               Sink &sink) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    AT p[J];
    int hd[J];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        hd[k] = is_head(R.col[k]);
        p[k] = (AT)R.v[k] * (AT)R.xv[k];
    }
    CSeg<AT> s{0, AT(0)};
#pragma unroll
    for (int k = 0; k < J; ++k) {
        s.v = hd[k] ? p[k] : s.v + p[k];
        s.c += hd[k];
    }
    s = wave_scan_dpp(s, CSegStep{});
    if (lane == kWave - 1) wave_tot[wid] = s;
    __syncthreads();
    CSeg<AT> pre = seed, total = seed;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const CSeg<AT> t = wave_tot[w];
        if (w < wid) pre = cseg_combine(pre, t);
        total = cseg_combine(total, t);
    }
    __syncthreads();
    const CSeg<AT> ex{shfl_up(s.c, 1), shfl_up(s.v, 1)};
    const CSeg<AT> in = lane == 0 ? pre : cseg_combine(pre, ex);
    AT acc = in.v;
    int cnt = in.c;
#pragma unroll
    for (int k = 0; k < J; ++k) {
        if (hd[k]) {
            if (cnt > 0) sink.row_done(cnt - 1, acc);
            acc = p[k];
            ++cnt;
        } else {
            acc += p[k];
        }
        sink.entry(cnt - 1, col_of(R.col[k]), R.v[k]);
    }
    return total;
}


// ------------------------------------------------------------------ BSS tile
// Output sink of the row-sum kernels: row r of the CSR goes to y[ridx[r]]
// (or y[r] when ridx is null).
template <class YT, class AT>
struct StoreSink {
    YT *y;
    const int32_t *ridx;  // row r of the CSR is output row ridx[r] (null: r itself)
    __device__ int64_t out(int32_t r) const { return ridx ? ridx[r] : r; }
    __device__ void row_done(int32_t r, AT v) { y[out(r)] = (YT)v; }
    __device__ void empty_row(int32_t r) { y[out(r)] = YT(0); }
    template <class VT>
    __device__ void entry(int32_t, int32_t, VT) {}
};

// One branchless segmented-scan tile (the BSS layout).
// Tile t = entries [tT, min((t+1)T, nnz)), T = 256 * J.  Rows that start
// and end in the tile are written directly.  The last row started in the
// tile, if it runs past the tile, leaves its partial in tail_val[t]; the
// leading partial of a row begun in an earlier tile goes to carry_val[t].
// The fix-up kernel then writes each such row once: its start partial plus
// the carries of the following tiles in ascending tile order.
template <int NT, class VT, class XT, class YT, class AT, int J>
__device__ __forceinline__ void bss_tile(int64_t t, const int32_t *__restrict__ rowptr,
                                         const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                         const XT *__restrict__ x, YT *__restrict__ y, int64_t nnz,
                                         const int32_t *__restrict__ row_lo, const int32_t *__restrict__ carry_row,
                                         AT *__restrict__ carry_val, AT *__restrict__ tail_val,
                                         int32_t *__restrict__ tail_row, int32_t *head_row, Seg<AT> *wave_tot,
                                         const int32_t *__restrict__ ridx) {
    constexpr int T = NT * J;
    const int64_t A = t * T;
    const int64_t c1 = (A + T < nnz) ? A + T : nnz;
    StoreSink<YT, AT> sink{y, ridx};
    // loads first; the row-pointer probe and the gathers overlap them
    Run<J, VT, XT> R;
    run_load<NT, J>(R, A, A, c1, colind, val);
    clear_heads<NT, J>(head_row);
    const int32_t rlo = row_lo[t], rend = row_lo[t + 1];
    const RowProbe probe = first_row<NT>(rowptr, rlo, rend);
    run_gather(R, x);
    __syncthreads();
    mark_rows<NT>(rowptr, probe, rlo, rend, A, A + T, true, head_row, sink);
    Seg<AT> seed{0, AT(0), -1};
    ChunkResult<AT> res = seg_chunk<NT, J, VT, XT, AT>(R, head_row, seed, wave_tot, sink);
    const int32_t cr = carry_row[t];
    if (res.has_lead && cr >= 0) carry_val[t] = res.lead;
    if (threadIdx.x == 0) {
        int32_t tr = -1;
        if (!res.state.f) {
            // no row starts in this tile: all of it belongs to the carried row
            if (cr >= 0) carry_val[t] = res.state.v;
        } else if (rowptr[res.state.r + 1] <= c1) {
            y[sink.out(res.state.r)] = (YT)res.state.v;
        } else {
            tr = res.state.r;
            tail_val[t] = res.state.v;
        }
        tail_row[t] = tr;
    }
}

}  // namespace xab
