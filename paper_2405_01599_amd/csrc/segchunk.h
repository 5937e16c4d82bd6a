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
// (written by mark_heads from rowptr; empty rows never start a segment).
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

// Mark row starts of rows [rlo, rhi) in head_row (indices relative to A);
// empty rows go to sink.empty_row.  head_row must hold -1 everywhere first.
template <int NT, class Sink>
__device__ __forceinline__ void mark_heads(const int32_t *__restrict__ rowptr, int32_t rlo, int32_t rhi, int64_t A,
                                           int32_t *head_row, Sink &sink) {
    for (int32_t r = rlo + (int32_t)threadIdx.x; r < rhi; r += NT) {
        int32_t q0 = rowptr[r], q1 = rowptr[r + 1];
        if (q1 > q0) head_row[q0 - A] = r;
        else sink.empty_row(r);
    }
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

template <int NT, int J, class VT, class XT, class AT, class Sink>
__device__ __forceinline__ ChunkResult<AT> seg_chunk(int64_t A, int64_t c0, int64_t c1,
                                                     const int32_t *__restrict__ colind,
                                                     const VT *__restrict__ val, const XT *__restrict__ x,
                                                     const int32_t *head_row, Seg<AT> seed, Seg<AT> *wave_tot,
                                                     Sink &sink) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int64_t base = A + (int64_t)tid * J;

    VT v[J];
    int32_t col[J];
    AT p[J];
    int32_t hr[J];
    if (base >= c0 && base + J <= c1) {
        load_run_full<VT, J>(val, base, v);
        load_run_full<int32_t, J>(colind, base, col);
#pragma unroll
        for (int k = 0; k < J; ++k) p[k] = (AT)v[k] * (AT)x[col[k]];
    } else {
#pragma unroll
        for (int k = 0; k < J; ++k) {
            int64_t q = base + k;
            bool live = q >= c0 && q < c1;
            v[k] = live ? __builtin_nontemporal_load(val + q) : VT(0);
            col[k] = live ? __builtin_nontemporal_load(colind + q) : -1;
            p[k] = live ? (AT)v[k] * (AT)x[col[k]] : AT(0);
        }
    }
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
        sink.entry(row, col[k], v[k]);
    }
    return res;
}

}  // namespace xab
