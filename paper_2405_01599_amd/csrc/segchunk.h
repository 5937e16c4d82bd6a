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

}  // namespace xab
