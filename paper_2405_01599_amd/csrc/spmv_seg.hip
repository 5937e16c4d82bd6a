// SpMV implementations built on the segmented chunk reduction:
//   nnz-split (the paper's non-zero elements based decomposition),
//   branchless segmented scan (with its carry fix-up),
//   symmetric SpMV with zero-element omission in the transpose reduction.
// The column-blocked variant lives in spmv_xcb.hip.
#include "segchunk.h"
#include "spmv_launch.h"
#include "sym_layout.h"

namespace xab {
namespace {

constexpr int kNT = 256;      // threads per workgroup
constexpr int kChunkJ = 8;    // entries per lane per chunk (nnz-split)

// ------------------------------------------------------------------ nnz-split
// Workgroup p owns whole rows [b[p], b[p+1]) (about T entries).  It walks
// them in chunks of 256*8 entries aligned to the chunk size; a row crossing
// a chunk boundary stays open in the scan seed, so every row is written
// exactly once, by the workgroup that owns it.
template <class VT, class XT, class YT, class AT>
__global__ __launch_bounds__(kNT) void k_spmv_nnz(const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                                  const XT *__restrict__ x, YT *__restrict__ y,
                                                  const int32_t *__restrict__ b, int64_t P) {
    constexpr int CH = kNT * kChunkJ;
    __shared__ int32_t head_row[CH];
    __shared__ Seg<AT> wave_tot[kNT / kWave];
    const int64_t p = xcd_remap(blockIdx.x, P);
    const int32_t r0 = b[p], r1 = b[p + 1];
    if (r0 >= r1) return;
    const int64_t s = rowptr[r0], e = rowptr[r1];
    StoreSink<YT, AT> sink{y, nullptr};
    Seg<AT> seed{0, AT(0), -1};
    int32_t rlo = r0;
    int64_t A = s - (s % CH);
    Run<kChunkJ, VT, XT> R;
    run_load<kNT, kChunkJ>(R, A, s, e < A + CH ? e : A + CH, colind, val);
    for (;;) {
        const int64_t Aend = A + CH;
        const bool last = Aend >= e;
        clear_heads<kNT, kChunkJ>(head_row);
        const RowProbe probe = first_row<kNT>(rowptr, rlo, r1);
        run_gather(R, x);
        __syncthreads();
        const int32_t rhi = mark_rows<kNT>(rowptr, probe, rlo, r1, A, Aend, last, head_row, sink);
        // the next chunk's loads fly while this one is scanned
        Run<kChunkJ, VT, XT> Rn;
        if (!last) run_load<kNT, kChunkJ>(Rn, Aend, Aend, e < Aend + CH ? e : Aend + CH, colind, val);
        ChunkResult<AT> res = seg_chunk<kNT, kChunkJ, VT, XT, AT>(R, head_row, seed, wave_tot, sink);
        seed = res.state;
        rlo = rhi;
        if (last) break;
        A = Aend;
        R = Rn;
    }
    if (threadIdx.x == 0 && seed.f) y[seed.r] = (YT)seed.v;
}

// ------------------------------------------------------------------ BSS
// (tile body bss_tile in segchunk.h)
template <class VT, class XT, class YT, class AT, int J>
__global__ __launch_bounds__(kNT) void k_spmv_bss(const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                                  const XT *__restrict__ x, YT *__restrict__ y, int64_t nnz,
                                                  int64_t P, const int32_t *__restrict__ row_lo,
                                                  const int32_t *__restrict__ carry_row, AT *__restrict__ carry_val,
                                                  AT *__restrict__ tail_val, int32_t *__restrict__ tail_row) {
    __shared__ int32_t head_row[kNT * J];
    __shared__ Seg<AT> wave_tot[kNT / kWave];
    bss_tile<kNT, VT, XT, YT, AT, J>(xcd_remap(blockIdx.x, P), rowptr, colind, val, x, y, nnz, row_lo, carry_row,
                                carry_val, tail_val, tail_row, head_row, wave_tot, nullptr);
}

template <class YT, class AT>
__global__ void k_bss_fixup(YT *__restrict__ y, int64_t P, const int32_t *__restrict__ carry_row,
                            const AT *__restrict__ carry_val, const AT *__restrict__ tail_val,
                            const int32_t *__restrict__ tail_row) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    int32_t r = tail_row[t];
    if (r < 0) return;
    AT acc = tail_val[t];
    for (int64_t u = t + 1; u < P && carry_row[u] == r; ++u) acc += carry_val[u];
    y[r] = (YT)acc;
}

// ------------------------------------------------------------------ symmetric S3
// y = (L + L_strict^T) x from the lower triangle L.  One wave per tile:
// tile p owns rows [b[p], b[p+1]) and walks their entries in chunks of
// 64 * kChunkJ (chunks start at multiples of that size), lane l holding
// kChunkJ consecutive entries.  Row sums come from the segmented scan.
// Every strictly-lower entry (i, j) adds L_ij x_i to row j: to the tile's
// accumulator of row j when j is one of its rows, else to j's slot in the
// tile's copy of column block j / C.  The touch map lists exactly the
// blocks a tile reaches; no other part of the reduction vector is ever
// read or written.  At the end the tile writes its rows of y and its block
// partials, and the block-reduce kernel adds, per touched block, the
// partials of the later tiles in ascending tile order.
//
// Fixed summation order: one wave issues every addition to the tile's
// accumulators, slot k of a chunk (entry k of each lane) in one LDS add
// instruction, slots in order, chunks in order.  The plan sets bit 30 of
// an entry in its column copy when a lower lane of the same slot adds to
// the same row; such entries are added after the chunk's slots, one lane
// at a time in lane order.  No two lanes of one add instruction meet on an
// address, so y is the same bit for bit on every run.
namespace symk {
constexpr int J = sym::kChunkJ;
constexpr int CH = sym::kChunk;

// tile-local slot of row j (j below the tile's row i): own row, or the
// row's place in the tile's copy of its column block
template <int C>
struct Slots {
    const int16_t *lut;
    int32_t r0, minblk, own_cap;
    __device__ __forceinline__ int at(int32_t j) const {
        if (j >= r0) return j - r0;
        return own_cap + (int)lut[j / C - minblk] * C + (j & (C - 1));
    }
};

template <class VT, class XT>
__device__ __forceinline__ void gather(Run<J, VT, XT> &R, const XT *__restrict__ x) {
#pragma unroll
    for (int k = 0; k < J; ++k)
        R.xv[k] = R.col[k] != kDeadCol ? x[(uint32_t)R.col[k] & sym::kColMask] : XT(0);
}

// the transposed part of one chunk: entry k of the lane lies in tile-local
// row rl[k] (-1: dead slot)
template <class VT, class XT, class AT, int C>
__device__ __forceinline__ void transpose_adds(const Run<J, VT, XT> &R, const int (&rl)[J], AT *acc, const AT *xs,
                                               const Slots<C> &sl) {
    AT xr[J];
#pragma unroll
    for (int k = 0; k < J; ++k) xr[k] = rl[k] >= 0 ? xs[rl[k]] : AT(0);
    int tg[J];
    int defer = 0;
#pragma unroll
    for (int k = 0; k < J; ++k) {
        const uint32_t c = (uint32_t)R.col[k];
        const int32_t j = (int32_t)(c & sym::kColMask);
        const bool live = R.col[k] != kDeadCol && rl[k] >= 0 && j < sl.r0 + rl[k];
        tg[k] = live ? sl.at(j) : -1;
        defer |= (live && (c & sym::kDeferBit)) ? 1 << k : 0;
    }
#pragma unroll
    for (int k = 0; k < J; ++k)
        if (tg[k] >= 0 && !((defer >> k) & 1)) atomicAdd(&acc[tg[k]], (AT)R.v[k] * xr[k]);
    uint64_t m = __ballot(defer != 0);
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        if ((int)threadIdx.x == l) {
#pragma unroll
            for (int k = 0; k < J; ++k)
                if ((defer >> k) & 1) atomicAdd(&acc[tg[k]], (AT)R.v[k] * xr[k]);
        }
    }
}

// one chunk of the flagged stream (every row of the tile non-empty): rows
// are counted from the tile's first head; `seed` = heads seen before the
// chunk and the open row's partial
template <class VT, class XT, class AT, int C>
__device__ __forceinline__ CSeg<AT> chunk_flagged(const Run<J, VT, XT> &R, CSeg<AT> seed, AT *acc, const AT *xs,
                                                  const Slots<C> &sl) {
    const int lane = threadIdx.x;
    AT p[J];
    int hd[J];
    CSeg<AT> s{0, AT(0)};
#pragma unroll
    for (int k = 0; k < J; ++k) {
        hd[k] = is_head(R.col[k]);
        p[k] = (AT)R.v[k] * (AT)R.xv[k];
        s.v = hd[k] ? p[k] : s.v + p[k];
        s.c += hd[k];
    }
    const CSeg<AT> inc = wave_scan_dpp(s, CSegStep{});
    const CSeg<AT> all{__shfl(inc.c, kWave - 1), __shfl(inc.v, kWave - 1)};
    const CSeg<AT> ex{shfl_up(inc.c, 1), shfl_up(inc.v, 1)};
    const CSeg<AT> in = lane == 0 ? seed : cseg_combine(seed, ex);
    AT a = in.v;
    int cnt = in.c;
    int rl[J];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        if (hd[k]) {
            if (cnt > 0) atomicAdd(&acc[cnt - 1], a);  // a row ends: distinct rows across lanes
            a = p[k];
            ++cnt;
        } else {
            a += p[k];
        }
        rl[k] = cnt - 1;
    }
    transpose_adds<VT, XT, AT, C>(R, rl, acc, xs, sl);
    return cseg_combine(seed, all);
}

// one chunk walked with row pointers (a tile with empty rows): head_row
// holds the row starting at each position of the chunk, or -1
template <class VT, class XT, class AT, int C>
__device__ __forceinline__ Seg<AT> chunk_rows(const Run<J, VT, XT> &R, const int32_t *head_row, Seg<AT> seed,
                                              AT *acc, const AT *xs, const Slots<C> &sl) {
    const int lane = threadIdx.x;
    AT p[J];
    int32_t hr[J];
    Seg<AT> s{0, AT(0), -1};
#pragma unroll
    for (int k = 0; k < J; ++k) {
        hr[k] = head_row[lane * J + k];
        p[k] = (AT)R.v[k] * (AT)R.xv[k];
        const int h = hr[k] >= 0;
        s.v = h ? p[k] : s.v + p[k];
        s.r = h ? hr[k] : s.r;
        s.f |= h;
    }
    const Seg<AT> inc = wave_seg_scan<AT>(s, lane);
    const Seg<AT> all{__shfl(inc.f, kWave - 1), __shfl(inc.v, kWave - 1), __shfl(inc.r, kWave - 1)};
    Seg<AT> ex;
    ex.f = shfl_up(inc.f, 1);
    ex.v = shfl_up(inc.v, 1);
    ex.r = shfl_up(inc.r, 1);
    const Seg<AT> in = lane == 0 ? seed : seg_combine(seed, ex);
    AT a = in.v;
    int32_t row = in.r;
    int open = in.f;
    int rl[J];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        if (hr[k] >= 0) {
            if (open) atomicAdd(&acc[row - sl.r0], a);
            a = p[k];
            row = hr[k];
            open = 1;
        } else {
            a += p[k];
        }
        rl[k] = open ? row - sl.r0 : -1;
    }
    transpose_adds<VT, XT, AT, C>(R, rl, acc, xs, sl);
    __syncthreads();  // head_row is cleared for the next chunk
    return seg_combine(seed, all);
}

struct NoSink {
    __device__ void empty_row(int32_t) {}
};

// sliced walk: up to G slots of a chunk per pass, lane = row (14: the
// lower triangle of a 27-point stencil row in one pass)
constexpr int G = 14;
constexpr int kSlWaves = 4;  // waves per tile workgroup: one chunk each per round
}  // namespace symk

template <class VT, class XT, class YT, class AT, int C>
__global__ __launch_bounds__(sym::kLanes) void k_spmv_sym_s3(
    const int32_t *__restrict__ rowptr, const VT *__restrict__ val, const XT *__restrict__ x, YT *__restrict__ y,
    const int32_t *__restrict__ b, int64_t P, const int32_t *__restrict__ tile_ptr,
    const int32_t *__restrict__ tile_blk, const int32_t *__restrict__ tile_slot,
    const int32_t *__restrict__ tile_minblk, AT *__restrict__ partial, int own_cap, int ext_cap,
    const int32_t *__restrict__ ci_f, const uint8_t *__restrict__ dense) {
    using namespace symk;
    extern __shared__ __align__(16) char smem[];
    AT *acc = (AT *)smem;                        // own rows [own_cap], then touched blocks [ext_cap]
    AT *xs = acc + own_cap + ext_cap;            // x of the own rows
    int32_t *head_row = (int32_t *)(xs + own_cap);  // [CH], tiles with empty rows
    int16_t *lut = (int16_t *)(head_row + CH);      // block id - minblk -> the tile's block index
    const int64_t p = xcd_remap(blockIdx.x, P);
    const int32_t r0 = b[p], r1 = b[p + 1];
    if (r0 >= r1) return;
    const int64_t s = rowptr[r0], e = rowptr[r1];
    const int32_t q0 = tile_ptr[p], nb = tile_ptr[p + 1] - q0;
    const Slots<C> sl{lut, r0, tile_minblk[p], own_cap};
    const int lane = threadIdx.x;
    for (int i = lane; i < r1 - r0; i += kWave) {
        acc[i] = AT(0);
        xs[i] = (AT)x[r0 + i];
    }
    for (int i = lane; i < nb * C; i += kWave) acc[own_cap + i] = AT(0);
    for (int i = lane; i < nb; i += kWave) lut[tile_blk[q0 + i] - sl.minblk] = (int16_t)i;
    __syncthreads();

    const int64_t A0 = s - (s % CH);
    if (dense[p]) {
        // every row of the tile has an entry: rows are found by counting the
        // heads of the flagged copy; the next chunk's loads and gathers are in
        // flight while one is scanned
        Run<J, VT, XT> R0, R1;
        run_load<kWave, J>(R0, A0, s, e < A0 + CH ? e : A0 + CH, ci_f, val);
        gather(R0, x);
        if (A0 + CH < e) run_load<kWave, J>(R1, A0 + CH, A0 + CH, e < A0 + 2 * CH ? e : A0 + 2 * CH, ci_f, val);
        CSeg<AT> st{0, AT(0)};
        for (int64_t A = A0;; A += CH) {
            const bool last = A + CH >= e;
            if (!last) gather(R1, x);
            Run<J, VT, XT> R2;
            if (A + 2 * CH < e)
                run_load<kWave, J>(R2, A + 2 * CH, A + 2 * CH, e < A + 3 * CH ? e : A + 3 * CH, ci_f, val);
            st = chunk_flagged<VT, XT, AT, C>(R0, st, acc, xs, sl);
            if (last) break;
            R0 = R1;
            R1 = R2;
        }
        if (lane == 0 && st.c > 0) atomicAdd(&acc[st.c - 1], st.v);
    } else {
        Seg<AT> seed{0, AT(0), -1};
        int32_t rlo = r0;
        int64_t A = A0;
        Run<J, VT, XT> R;
        NoSink ns;
        run_load<kWave, J>(R, A, s, e < A + CH ? e : A + CH, ci_f, val);
        for (;;) {
            const int64_t Aend = A + CH;
            const bool last = Aend >= e;
            clear_heads<kWave, J>(head_row);
            const RowProbe probe = first_row<kWave>(rowptr, rlo, r1);
            gather(R, x);
            __syncthreads();
            const int32_t rhi = mark_rows<kWave>(rowptr, probe, rlo, r1, A, Aend, last, head_row, ns);
            Run<J, VT, XT> Rn;
            if (!last) run_load<kWave, J>(Rn, Aend, Aend, e < Aend + CH ? e : Aend + CH, ci_f, val);
            seed = chunk_rows<VT, XT, AT, C>(R, head_row, seed, acc, xs, sl);
            rlo = rhi;
            if (last) break;
            A = Aend;
            R = Rn;
        }
        if (lane == 0 && seed.f) atomicAdd(&acc[seed.r - r0], seed.v);
    }
    __syncthreads();
    for (int i = lane; i < r1 - r0; i += kWave) y[r0 + i] = (YT)acc[i];
    for (int i = lane; i < nb * C; i += kWave) {
        const int q = i / C;
        partial[(int64_t)tile_slot[q0 + q] * C + (i % C)] = acc[own_cap + i];
    }
}

// The sliced walk of the symmetric product (the plan's padded copy, lane =
// row): tile p's rows in chunks of 64, each chunk column-major with stride
// = its row count.  Four waves per tile take the chunks in rounds (wave w
// takes chunk 4r + w) and walk up to G slots of their chunk per pass: each
// lane loads its slots, gathers x, sums its row serially (slots in order)
// and forms the transposed products of its strictly-lower entries.  The
// additions to the tile's accumulators then happen wave by wave (barriers
// between), slot by slot, one LDS add instruction per slot; the entries
// the plan marks with bit 30 (a lower lane of the same slot meets the same
// row) follow the wave's slots, lane by lane; a chunk's row sums follow its
// last pass.  So the order of every addition is fixed by the plan.  Adds
// that add nothing (dead slots, entries on the diagonal, deferred entries,
// lanes past the chunk's rows) go to a spare slot per lane, so no add is
// branched around, and every lane issues every load (a dead slot reads the
// chunk's first entry), so the waits count the loads in flight exactly.
template <class VT, class XT, class YT, class AT, int C>
__global__ __launch_bounds__(sym::kLanes * symk::kSlWaves) void k_spmv_sym_sliced(
    const XT *__restrict__ x, YT *__restrict__ y, const int32_t *__restrict__ b, int64_t P,
    const int32_t *__restrict__ tile_ptr, const int32_t *__restrict__ tile_blk,
    const int32_t *__restrict__ tile_slot, const int32_t *__restrict__ tile_minblk, AT *__restrict__ partial,
    int own_cap, int ext_cap, int lut_cap, const int32_t *__restrict__ ch0, const int32_t *__restrict__ cw,
    const int64_t *__restrict__ coff, const int32_t *__restrict__ cols, const VT *__restrict__ vals) {
    using namespace symk;
    constexpr int NT = sym::kLanes * kSlWaves;
    extern __shared__ __align__(16) char smem[];
    AT *acc = (AT *)smem;  // own rows [own_cap], touched blocks [ext_cap], a spare slot per lane
    int16_t *lut = (int16_t *)(acc + own_cap + ext_cap + kWave);
    const int64_t p = xcd_remap(blockIdx.x, P);
    const int32_t r0 = b[p], r1 = b[p + 1];
    if (r0 >= r1) return;
    const int32_t q0 = tile_ptr[p], nb = tile_ptr[p + 1] - q0;
    const int32_t minblk = tile_minblk[p];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int32_t g0 = ch0[p];
    const int nct = ch0[p + 1] - g0;
    for (int i = tid; i < r1 - r0; i += NT) acc[i] = AT(0);
    for (int i = tid; i < nb * C; i += NT) acc[own_cap + i] = AT(0);
    for (int i = tid; i < nb; i += NT) lut[tile_blk[q0 + i] - minblk] = (int16_t)i;
    __syncthreads();
    const int trash = own_cap + ext_cap + lane;
    for (int c0 = 0; c0 < nct; c0 += kSlWaves) {
        // this wave's chunk of the round (none past the tile's last)
        const int c = c0 + wid;
        const bool has = c < nct;
        const int32_t rc = r0 + kWave * c;
        const int nr = has ? min(kWave, r1 - rc) : 0;
        const int w = has ? cw[g0 + c] : 0;
        const int64_t o = has ? coff[g0 + c] : 0;
        // passes of the round: enough for its widest chunk (one for empty ones)
        int wmax = 1;
        for (int u = 0; u < kSlWaves && c0 + u < nct; ++u) wmax = max(wmax, cw[g0 + c0 + u]);
        const bool on = lane < nr;
        const int32_t i = rc + lane;
        const XT xr = x[on ? (uint32_t)i : 0u];
        const AT xi = on ? (AT)xr : AT(0);
        AT rs = AT(0);
        for (int k0 = 0; k0 < wmax; k0 += G) {
            int32_t cc[G];
            VT v[G];
            uint32_t off = (uint32_t)(k0 * nr + lane);
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const bool live = on && k0 + u < w;
                const uint32_t q = live ? off : 0u;
                const int32_t cv = __builtin_nontemporal_load(cols + o + q);
                const VT vv = __builtin_nontemporal_load(vals + o + q);
                cc[u] = live ? cv : kDeadCol;
                v[u] = live ? vv : VT(0);
                off += (uint32_t)nr;
            }
            XT xv[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const bool live = cc[u] != kDeadCol;
                const XT g = x[live ? ((uint32_t)cc[u] & sym::kColMask) : 0u];  // a dead slot reads x[0]
                xv[u] = live ? g : XT(0);
            }
            int tg[G];
            int defer = 0, now = 0;
#pragma unroll
            for (int u = 0; u < G; ++u) {
                rs += (AT)v[u] * (AT)xv[u];
                const int32_t j = (int32_t)((uint32_t)cc[u] & sym::kColMask);
                const int32_t d = j / C - minblk;  // every lookup in range, needed or not
                const int16_t lb = lut[d < 0 ? 0 : (d >= lut_cap ? lut_cap - 1 : d)];
                const bool live = cc[u] != kDeadCol && j < i;
                const bool nw = live && !((uint32_t)cc[u] & sym::kDeferBit);
                tg[u] = j >= r0 ? j - r0 : own_cap + (int)lb * C + (j & (C - 1));
                defer |= (live && !nw) ? 1 << u : 0;
                now |= nw ? 1 << u : 0;
            }
            const bool last = k0 + G >= wmax;
            // the adds, wave by wave: each wave's adds complete (the wait on
            // the LDS counter) before the barrier lets the next wave add
            for (int ww = 0; ww < kSlWaves; ++ww) {
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                __syncthreads();
                if (wid == ww) {
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const bool nw = (now >> u) & 1;
                        atomicAdd(&acc[nw ? tg[u] : trash], nw ? (AT)v[u] * xi : AT(0));
                    }
                    uint64_t m = __ballot(defer != 0);
                    while (m) {
                        const int l = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        if (lane == l) {
#pragma unroll
                            for (int u = 0; u < G; ++u)
                                if ((defer >> u) & 1) atomicAdd(&acc[tg[u]], (AT)v[u] * xi);
                        }
                    }
                    if (last) atomicAdd(&acc[on ? i - r0 : trash], on ? rs : AT(0));
                }
            }
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
    for (int r = tid; r < r1 - r0; r += NT) y[r0 + r] = (YT)acc[r];
    for (int r = tid; r < nb * C; r += NT) {
        const int q = r / C;
        partial[(int64_t)tile_slot[q0 + q] * C + (r % C)] = acc[own_cap + r];
    }
}

// Adds to each row of a touched column block the partials of the tiles
// listed for that block, in the listed (ascending tile) order.
template <class YT, class AT, int C>
__global__ void k_sym_block_reduce(YT *__restrict__ y, int32_t n, const int32_t *__restrict__ tm_ptr,
                                   const AT *__restrict__ partial) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int64_t c = j / C;
    int32_t s0 = tm_ptr[c], s1 = tm_ptr[c + 1];
    if (s0 == s1) return;
    AT acc = AT(0);
    for (int32_t s = s0; s < s1; ++s) acc += partial[(int64_t)s * C + (j % C)];
    y[j] = (YT)((AT)y[j] + acc);
}

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <class VT, class XT, class YT, class AT>
int launch_nnz(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    hipLaunchKernelGGL((k_spmv_nnz<VT, XT, YT, AT>), dim3((unsigned)pl->P), dim3(kNT), 0, ctx->stream, A->rowptr,
                       A->colind, val, x, y, pl->b, pl->P);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_nnz");
    return XAB_OK;
}

template <class VT, class XT, class YT, class AT, int J>
static int launch_bss_j(xab_ctx *ctx, const BssArgs &a, const VT *val, const XT *x, YT *y) {
    hipLaunchKernelGGL((k_spmv_bss<VT, XT, YT, AT, J>), dim3((unsigned)a.P), dim3(kNT), 0, ctx->stream, a.rowptr,
                       a.colind, val, x, y, a.nnz, a.P, a.row_lo, a.carry_row, (AT *)a.carry_val, (AT *)a.tail_val,
                       a.tail_row);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_bss");
    hipLaunchKernelGGL((k_bss_fixup<YT, AT>), dim3(grid_for(a.P, 256)), dim3(256), 0, ctx->stream, y, a.P,
                       a.carry_row, (const AT *)a.carry_val, (const AT *)a.tail_val, a.tail_row);
    XAB_LAUNCH_CHECK(ctx, "k_bss_fixup");
    return XAB_OK;
}

template <class VT, class XT, class YT, class AT>
int launch_bss_raw(xab_ctx *ctx, const BssArgs &a, const VT *val, const XT *x, YT *y) {
    switch (a.j) {
        case 1: return launch_bss_j<VT, XT, YT, AT, 1>(ctx, a, val, x, y);
        case 2: return launch_bss_j<VT, XT, YT, AT, 2>(ctx, a, val, x, y);
        case 4: return launch_bss_j<VT, XT, YT, AT, 4>(ctx, a, val, x, y);
        case 8: return launch_bss_j<VT, XT, YT, AT, 8>(ctx, a, val, x, y);
        case 16: return launch_bss_j<VT, XT, YT, AT, 16>(ctx, a, val, x, y);
        case 32: return launch_bss_j<VT, XT, YT, AT, 32>(ctx, a, val, x, y);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane %d", a.j);
    }
}

template <class VT, class XT, class YT, class AT>
int launch_bss(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const BssArgs a{pl->A->rowptr, pl->A->colind, pl->A->nnz, pl->P, pl->params.j_per_lane, pl->row_lo,
                    pl->carry_row, pl->carry_val, pl->tail_val, pl->tail_row};
    return launch_bss_raw<VT, XT, YT, AT>(ctx, a, val, x, y);
}

template <class VT, class XT, class YT, class AT, int C>
static int launch_s3_c(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    const size_t lds = sym::lds_bytes(pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap, (int)sizeof(AT));
    if (lds > (size_t)sym::kLdsCap)
        return xab_fail(ctx, XAB_E_UNSUPPORTED, "symmetric tile needs %zu bytes of LDS", lds);
    if (pl->s3_walk) {
        const VT *pv;
        if constexpr (sizeof(VT) == 8) pv = (const VT *)pl->s3_v64;
        else pv = (const VT *)pl->s3_v32;
        if (!pv) return xab_fail(ctx, XAB_E_DTYPE, "the plan's sliced copy holds no values of this precision");
        const size_t lds_sl = sym::lds_sliced(pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap, (int)sizeof(AT));
        hipLaunchKernelGGL((k_spmv_sym_sliced<VT, XT, YT, AT, C>), dim3((unsigned)pl->P),
                           dim3(sym::kLanes * symk::kSlWaves), lds_sl,
                           ctx->stream, x, y, pl->b, pl->P, pl->tile_ptr, pl->tile_blk, pl->tile_slot, pl->tile_minblk,
                           (AT *)pl->partial, pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap, pl->s3_ch0, pl->s3_cw,
                           pl->s3_coff, pl->s3_cols, pv);
        XAB_LAUNCH_CHECK(ctx, "k_spmv_sym_sliced");
    } else {
        hipLaunchKernelGGL((k_spmv_sym_s3<VT, XT, YT, AT, C>), dim3((unsigned)pl->P), dim3(sym::kLanes), lds,
                           ctx->stream, A->rowptr, val, x, y, pl->b, pl->P, pl->tile_ptr, pl->tile_blk,
                           pl->tile_slot, pl->tile_minblk, (AT *)pl->partial, pl->s3_own_cap, pl->s3_ext_cap,
                           pl->s3_ci, pl->s3_dense);
        XAB_LAUNCH_CHECK(ctx, "k_spmv_sym_s3");
    }
    if (pl->ntouch > 0) {
        hipLaunchKernelGGL((k_sym_block_reduce<YT, AT, C>), dim3(grid_for(A->n, 256)), dim3(256), 0, ctx->stream, y,
                           A->n, pl->tm_ptr, (const AT *)pl->partial);
        XAB_LAUNCH_CHECK(ctx, "k_sym_block_reduce");
    }
    return XAB_OK;
}

// A tile's accumulators live in LDS and take one atomic add per stored
// entry.  On gfx950 the return-less FP32 LDS atomic add runs about 20x
// slower than the FP64 one (3.2 vs 72 G wave instructions/s with distinct
// consecutive addresses), so the symmetric product accumulates in FP64
// whatever accumulation type is asked for: FP32 accumulation gives the
// FP64-accumulation result, at its speed (27-point 128^3 stencil, FP32
// values: 201 -> 80 us).
template <class VT, class XT, class YT, class AT>
int launch_sym_s3(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    using LT = double;
    switch (pl->params.col_block) {
        case 16: return launch_s3_c<VT, XT, YT, LT, 16>(ctx, pl, val, x, y);
        case 32: return launch_s3_c<VT, XT, YT, LT, 32>(ctx, pl, val, x, y);
        case 64: return launch_s3_c<VT, XT, YT, LT, 64>(ctx, pl, val, x, y);
        case 128: return launch_s3_c<VT, XT, YT, LT, 128>(ctx, pl, val, x, y);
        case 256: return launch_s3_c<VT, XT, YT, LT, 256>(ctx, pl, val, x, y);
        case 512: return launch_s3_c<VT, XT, YT, LT, 512>(ctx, pl, val, x, y);
        case 1024: return launch_s3_c<VT, XT, YT, LT, 1024>(ctx, pl, val, x, y);
        case 2048: return launch_s3_c<VT, XT, YT, LT, 2048>(ctx, pl, val, x, y);
        case 4096: return launch_s3_c<VT, XT, YT, LT, 4096>(ctx, pl, val, x, y);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "col_block %d", pl->params.col_block);
    }
}

XAB_INSTANTIATE_LAUNCHER(launch_nnz)
XAB_INSTANTIATE_LAUNCHER(launch_bss)
template int launch_bss_raw<double, double, double, double>(xab_ctx *, const BssArgs &, const double *,
                                                            const double *, double *);
template int launch_bss_raw<float, float, float, float>(xab_ctx *, const BssArgs &, const float *, const float *,
                                                        float *);
template int launch_bss_raw<float, float, float, double>(xab_ctx *, const BssArgs &, const float *, const float *,
                                                         float *);
template int launch_bss_raw<float, float, double, double>(xab_ctx *, const BssArgs &, const float *, const float *,
                                                          double *);
XAB_INSTANTIATE_LAUNCHER(launch_sym_s3)

}  // namespace xab
