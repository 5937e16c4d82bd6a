// SpMV implementations built on the segmented chunk reduction:
//   nnz-split (the paper's non-zero elements based decomposition),
//   branchless segmented scan (with its carry fix-up),
//   symmetric SpMV with zero-element omission in the transpose reduction.
#include "segchunk.h"
#include "spmv_launch.h"
#include "sym_layout.h"

namespace xab {
namespace {

constexpr int kNT = 256;      // threads per workgroup
constexpr int kChunkJ = 8;    // entries per lane per chunk (nnz-split)
constexpr int kSymJ = 4;      // entries per lane per chunk (symmetric: keeps v and col live)

// dynamic LDS layout of the symmetric kernel: heads, wave totals, then
// own[own_cap], ext[ext_cap] (accumulation type), lut[lut_cap] (int16)
__host__ __device__ constexpr int sym_off_wave() { return kNT * kSymJ * 4; }
template <class AT>
__host__ __device__ constexpr int sym_off_own() {
    return (sym_off_wave() + (kNT / kWave) * (int)sizeof(Seg<AT>) + 15) / 16 * 16;
}
template <class AT>
size_t sym_lds_bytes(int own_cap, int ext_cap, int lut_cap) {
    return (size_t)sym_off_own<AT>() + sizeof(AT) * (2 * (size_t)own_cap + ext_cap) + 2 * (size_t)lut_cap;
}

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
// Tile t = entries [tT, min((t+1)T, nnz)), T = 256 * J.  Rows that start
// and end in the tile are written directly.  The last row started in the
// tile, if it runs past the tile, leaves its partial in tail_val[t]; the
// leading partial of a row begun in an earlier tile goes to carry_val[t].
// The fix-up kernel then writes each such row once: its start partial plus
// the carries of the following tiles in ascending tile order.
template <class VT, class XT, class YT, class AT, int J>
__device__ __forceinline__ void bss_tile(int64_t t, const int32_t *__restrict__ rowptr,
                                         const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                         const XT *__restrict__ x, YT *__restrict__ y, int64_t nnz,
                                         const int32_t *__restrict__ row_lo, const int32_t *__restrict__ carry_row,
                                         AT *__restrict__ carry_val, AT *__restrict__ tail_val,
                                         int32_t *__restrict__ tail_row, int32_t *head_row, Seg<AT> *wave_tot,
                                         const int32_t *__restrict__ ridx) {
    constexpr int T = kNT * J;
    const int64_t A = t * T;
    const int64_t c1 = (A + T < nnz) ? A + T : nnz;
    StoreSink<YT, AT> sink{y, ridx};
    // loads first; the row-pointer probe and the gathers overlap them
    Run<J, VT, XT> R;
    run_load<kNT, J>(R, A, A, c1, colind, val);
    clear_heads<kNT, J>(head_row);
    const int32_t rlo = row_lo[t], rend = row_lo[t + 1];
    const RowProbe probe = first_row<kNT>(rowptr, rlo, rend);
    run_gather(R, x);
    __syncthreads();
    mark_rows<kNT>(rowptr, probe, rlo, rend, A, A + T, true, head_row, sink);
    Seg<AT> seed{0, AT(0), -1};
    ChunkResult<AT> res = seg_chunk<kNT, J, VT, XT, AT>(R, head_row, seed, wave_tot, sink);
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

template <class VT, class XT, class YT, class AT, int J>
__global__ __launch_bounds__(kNT) void k_spmv_bss(const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                                  const XT *__restrict__ x, YT *__restrict__ y, int64_t nnz,
                                                  int64_t P, const int32_t *__restrict__ row_lo,
                                                  const int32_t *__restrict__ carry_row, AT *__restrict__ carry_val,
                                                  AT *__restrict__ tail_val, int32_t *__restrict__ tail_row) {
    __shared__ int32_t head_row[kNT * J];
    __shared__ Seg<AT> wave_tot[kNT / kWave];
    bss_tile<VT, XT, YT, AT, J>(xcd_remap(blockIdx.x, P), rowptr, colind, val, x, y, nnz, row_lo, carry_row,
                                carry_val, tail_val, tail_row, head_row, wave_tot, nullptr);
}

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
// Tile t of block k covers entries [tT, tT + T).  Its first entry lies in
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

// a live flagged column is never -1: flagged values are INT_MIN + col with
// col < 2^31 - 1, so -1 marks the dead slots past the end of a block
constexpr int32_t kDeadCol = -1;

template <class VT, class XT, class AT, int J>
__global__ __launch_bounds__(kNT) void k_spmv_xcb(XcbArgs a, const XT *__restrict__ x) {
    constexpr int T = kNT * J;
    constexpr int NW = kNT / kWave;
    __shared__ CSeg<AT> wave_tot[NW];
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
    if (base + J <= c1) {
        load_run_full<int32_t, J>(ci, base, cr);
        load_run_full<VT, J>(va, base, v);
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
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        CSeg<AT> u{shfl_up(s.c, d), shfl_up(s.v, d)};
        if (lane >= d) s = cseg_combine(u, s);
    }
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
    // before it > 0) or the carried-in row's part in this tile
    AT acc = in.v;
    int cnt = in.c;
#pragma unroll
    for (int q = 0; q < J; ++q) {
        if (hd[q]) {
            if (cnt > 0) Y[r0 + cnt] = acc;
            else if (!h0) ((AT *)a.carry_val[k])[t] = acc;
            acc = p[q];
            ++cnt;
        } else {
            acc += p[q];
        }
    }
    if (tid == 0) {
        int32_t tr = -1;
        if (total.c == 0) {
            // no row starts in the tile: all of it belongs to the carried row
            ((AT *)a.carry_val[k])[t] = total.v;
        } else if (hnext) {
            Y[r0 + total.c] = total.v;
        } else {
            tr = r0 + total.c;
            ((AT *)a.tail_val[k])[t] = total.v;
        }
        a.tail_row[k][t] = tr;
    }
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
template <class YT, class AT>
__global__ __launch_bounds__(kNT) void k_xcb_combine(XcbArgs a, const uint8_t *__restrict__ mask,
                                                     const int32_t *__restrict__ gbase, int64_t G, int64_t n,
                                                     YT *__restrict__ y) {
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
    AT acc = AT(0);
#pragma unroll
    for (int k = 0; k < kXcds; ++k) {
        if ((m >> k) & 1u) {
            int64_t off = (int64_t)gbase[(int64_t)k * (G + 1) + g] + pre[k];
            for (int q = 0; q < w; ++q) off += wcnt[k][q];
            acc += ((const AT *)a.Y[k])[off];
        }
    }
    y[i] = (YT)acc;
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
// y = (L + L_strict^T) x from the lower triangle L.  Tile p owns rows
// [b[p], b[p+1]) (at most kRowCap).  Its row sums and the transposed
// entries that land on its own rows accumulate in LDS (own[]).  Transposed
// entries landing below the tile (column j < b[p]) accumulate in LDS slots
// of the column blocks the touch map lists for the tile (ext[]); every
// other region of the reduction vector is known to be zero and is never
// touched.  At the end the tile writes its rows of y and its block
// partials; the block-reduce kernel adds, per touched block, the partials
// of the later tiles in ascending tile order.
// LDS is sized per plan (dynamic shared memory): own_cap = most rows in a
// tile, ext_cap = most touched blocks in a tile times C, lut_cap = widest
// span of touched block ids in a tile.
template <class VT, class XT, class YT, class AT, int C>
__global__ __launch_bounds__(kNT) void k_spmv_sym_s3(const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                                     const XT *__restrict__ x, YT *__restrict__ y,
                                                     const int32_t *__restrict__ b, int64_t P,
                                                     const int32_t *__restrict__ tile_ptr,
                                                     const int32_t *__restrict__ tile_blk,
                                                     const int32_t *__restrict__ tile_slot,
                                                     const int32_t *__restrict__ tile_minblk,
                                                     AT *__restrict__ partial, int own_cap, int ext_cap,
                                                     int lut_cap) {
    constexpr int CH = kNT * kSymJ;
    extern __shared__ __align__(16) char smem[];
    int32_t *head_row = (int32_t *)smem;
    Seg<AT> *wave_tot = (Seg<AT> *)(smem + sym_off_wave());
    AT *own = (AT *)(smem + sym_off_own<AT>());
    AT *xs = own + own_cap;  // x of the tile's own rows
    AT *ext = xs + own_cap;
    int16_t *lut = (int16_t *)(ext + ext_cap);
    const int64_t p = xcd_remap(blockIdx.x, P);
    const int32_t r0 = b[p], r1 = b[p + 1];
    if (r0 >= r1) return;
    const int64_t s = rowptr[r0], e = rowptr[r1];
    const int32_t q0 = tile_ptr[p], q1 = tile_ptr[p + 1];
    const int32_t nb = q1 - q0;
    const int32_t minblk = tile_minblk[p];
    const int tid = threadIdx.x;
    for (int i = tid; i < r1 - r0; i += kNT) {
        own[i] = AT(0);
        xs[i] = (AT)x[r0 + i];
    }
    for (int i = tid; i < nb * C; i += kNT) ext[i] = AT(0);
    for (int i = tid; i < lut_cap; i += kNT) lut[i] = 0;
    __syncthreads();
    for (int i = tid; i < nb; i += kNT) lut[tile_blk[q0 + i] - minblk] = (int16_t)i;

    struct Sink {
        AT *own;
        AT *ext;
        const int16_t *lut;
        const AT *xs;
        int32_t r0, minblk;
        __device__ void row_done(int32_t r, AT v) { atomicAdd(&own[r - r0], v); }
        __device__ void empty_row(int32_t) {}
        __device__ void entry(int32_t row, int32_t j, VT v) {
            if (j < 0 || j >= row) return;  // dead slot or diagonal
            AT tv = (AT)v * xs[row - r0];
            if (j >= r0) atomicAdd(&own[j - r0], tv);
            else atomicAdd(&ext[(int)lut[j / C - minblk] * C + (j % C)], tv);
        }
    } sink{own, ext, lut, xs, r0, minblk};

    Seg<AT> seed{0, AT(0), -1};
    int32_t rlo = r0;
    int64_t A = s - (s % CH);
    Run<kSymJ, VT, XT> R;
    run_load<kNT, kSymJ>(R, A, s, e < A + CH ? e : A + CH, colind, val);
    for (;;) {
        const int64_t Aend = A + CH;
        const bool last = Aend >= e;
        clear_heads<kNT, kSymJ>(head_row);
        const RowProbe probe = first_row<kNT>(rowptr, rlo, r1);
        run_gather(R, x);
        __syncthreads();
        const int32_t rhi = mark_rows<kNT>(rowptr, probe, rlo, r1, A, Aend, last, head_row, sink);
        Run<kSymJ, VT, XT> Rn;
        if (!last) run_load<kNT, kSymJ>(Rn, Aend, Aend, e < Aend + CH ? e : Aend + CH, colind, val);
        ChunkResult<AT> res = seg_chunk<kNT, kSymJ, VT, XT, AT>(R, head_row, seed, wave_tot, sink);
        seed = res.state;
        rlo = rhi;
        if (last) break;
        A = Aend;
        R = Rn;
    }
    if (tid == 0 && seed.f) atomicAdd(&own[seed.r - r0], seed.v);
    __syncthreads();
    for (int i = tid; i < r1 - r0; i += kNT) y[r0 + i] = (YT)own[i];
    for (int i = tid; i < nb * C; i += kNT) {
        int q = i / C;
        partial[(int64_t)tile_slot[q0 + q] * C + (i % C)] = ext[i];
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
static int launch_bss_j(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    hipLaunchKernelGGL((k_spmv_bss<VT, XT, YT, AT, J>), dim3((unsigned)pl->P), dim3(kNT), 0, ctx->stream, A->rowptr,
                       A->colind, val, x, y, A->nnz, pl->P, pl->row_lo, pl->carry_row, (AT *)pl->carry_val,
                       (AT *)pl->tail_val, pl->tail_row);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_bss");
    hipLaunchKernelGGL((k_bss_fixup<YT, AT>), dim3(grid_for(pl->P, 256)), dim3(256), 0, ctx->stream, y, pl->P,
                       pl->carry_row, (const AT *)pl->carry_val, (const AT *)pl->tail_val, pl->tail_row);
    XAB_LAUNCH_CHECK(ctx, "k_bss_fixup");
    return XAB_OK;
}

template <class VT, class XT, class YT, class AT>
int launch_bss(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    switch (pl->params.j_per_lane) {
        case 1: return launch_bss_j<VT, XT, YT, AT, 1>(ctx, pl, val, x, y);
        case 2: return launch_bss_j<VT, XT, YT, AT, 2>(ctx, pl, val, x, y);
        case 4: return launch_bss_j<VT, XT, YT, AT, 4>(ctx, pl, val, x, y);
        case 8: return launch_bss_j<VT, XT, YT, AT, 8>(ctx, pl, val, x, y);
        case 16: return launch_bss_j<VT, XT, YT, AT, 16>(ctx, pl, val, x, y);
        case 32: return launch_bss_j<VT, XT, YT, AT, 32>(ctx, pl, val, x, y);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane %d", pl->params.j_per_lane);
    }
}

template <class VT, class XT, class YT, class AT, int J>
static int launch_xcb_j(xab_ctx *ctx, const xab_plan *pl, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    constexpr int KB = xab_plan::kXcb;
    static_assert(KB == kXcds, "one column block per XCD");
    const int64_t n = A->n;
    if (n == 0) return XAB_OK;
    XcbArgs a;
    int64_t pmax = 1;
    AT *Y = (AT *)pl->xcb_Y;
    for (int k = 0; k < KB; ++k) {
        const int64_t b = pl->xcb_base[k], o = pl->xcb_toff[k];
        a.colind[k] = pl->xcb_colind + b;
        if constexpr (sizeof(VT) == 8) a.val[k] = pl->xcb_val64 + b;
        else a.val[k] = pl->xcb_val32 + b;
        a.row0[k] = pl->xcb_tile_row + o;
        a.carry_row[k] = pl->xcb_carry_row + o;
        a.tail_row[k] = pl->xcb_tail_row + o;
        a.carry_val[k] = (AT *)pl->xcb_carry_val + o;
        a.tail_val[k] = (AT *)pl->xcb_tail_val + o;
        a.Y[k] = Y + pl->xcb_ybase[k];
        a.nnz[k] = pl->xcb_base[k + 1] - b;
        a.P[k] = pl->xcb_P[k];
        pmax = std::max(pmax, pl->xcb_P[k]);
    }
    hipLaunchKernelGGL((k_spmv_xcb<VT, XT, AT, J>), dim3((unsigned)(KB * pmax)), dim3(kNT), 0, ctx->stream, a, x);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_xcb");
    hipLaunchKernelGGL((k_xcb_fixup<AT>), dim3(grid_for(KB * pmax, 256)), dim3(256), 0, ctx->stream, a, pmax);
    XAB_LAUNCH_CHECK(ctx, "k_xcb_fixup");
    hipLaunchKernelGGL((k_xcb_combine<YT, AT>), dim3((unsigned)pl->xcb_G), dim3(kNT), 0, ctx->stream, a,
                       pl->xcb_mask, pl->xcb_gbase, pl->xcb_G, n, y);
    XAB_LAUNCH_CHECK(ctx, "k_xcb_combine");
    return XAB_OK;
}

template <class VT, class XT, class YT, class AT>
int launch_xcb(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    (void)val;  // the plan holds its own column-blocked copy of the values
    if ((sizeof(VT) == 8 && !pl->xcb_val64) || (sizeof(VT) == 4 && !pl->xcb_val32))
        return xab_fail(ctx, XAB_E_DTYPE, "column-blocked plan holds no values of this precision");
    switch (pl->params.j_per_lane) {
        case 1: return launch_xcb_j<VT, XT, YT, AT, 1>(ctx, pl, x, y);
        case 2: return launch_xcb_j<VT, XT, YT, AT, 2>(ctx, pl, x, y);
        case 4: return launch_xcb_j<VT, XT, YT, AT, 4>(ctx, pl, x, y);
        case 8: return launch_xcb_j<VT, XT, YT, AT, 8>(ctx, pl, x, y);
        case 16: return launch_xcb_j<VT, XT, YT, AT, 16>(ctx, pl, x, y);
        case 32: return launch_xcb_j<VT, XT, YT, AT, 32>(ctx, pl, x, y);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane %d", pl->params.j_per_lane);
    }
}

template <class VT, class XT, class YT, class AT, int C>
static int launch_s3_c(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    const xab_matrix *A = pl->A;
    const size_t lds = sym_lds_bytes<AT>(pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap);
    if (lds > (size_t)sym::kLdsCap)
        return xab_fail(ctx, XAB_E_UNSUPPORTED, "symmetric tile needs %zu bytes of LDS", lds);
    hipLaunchKernelGGL((k_spmv_sym_s3<VT, XT, YT, AT, C>), dim3((unsigned)pl->P), dim3(kNT), lds, ctx->stream,
                       A->rowptr, A->colind, val, x, y, pl->b, pl->P, pl->tile_ptr, pl->tile_blk, pl->tile_slot,
                       pl->tile_minblk, (AT *)pl->partial, pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap);
    XAB_LAUNCH_CHECK(ctx, "k_spmv_sym_s3");
    if (pl->ntouch > 0) {
        hipLaunchKernelGGL((k_sym_block_reduce<YT, AT, C>), dim3(grid_for(A->n, 256)), dim3(256), 0, ctx->stream, y,
                           A->n, pl->tm_ptr, (const AT *)pl->partial);
        XAB_LAUNCH_CHECK(ctx, "k_sym_block_reduce");
    }
    return XAB_OK;
}

template <class VT, class XT, class YT, class AT>
int launch_sym_s3(xab_ctx *ctx, const xab_plan *pl, const VT *val, const XT *x, YT *y) {
    switch (pl->params.col_block) {
        case 16: return launch_s3_c<VT, XT, YT, AT, 16>(ctx, pl, val, x, y);
        case 32: return launch_s3_c<VT, XT, YT, AT, 32>(ctx, pl, val, x, y);
        case 64: return launch_s3_c<VT, XT, YT, AT, 64>(ctx, pl, val, x, y);
        case 128: return launch_s3_c<VT, XT, YT, AT, 128>(ctx, pl, val, x, y);
        case 256: return launch_s3_c<VT, XT, YT, AT, 256>(ctx, pl, val, x, y);
        case 512: return launch_s3_c<VT, XT, YT, AT, 512>(ctx, pl, val, x, y);
        case 1024: return launch_s3_c<VT, XT, YT, AT, 1024>(ctx, pl, val, x, y);
        case 2048: return launch_s3_c<VT, XT, YT, AT, 2048>(ctx, pl, val, x, y);
        case 4096: return launch_s3_c<VT, XT, YT, AT, 4096>(ctx, pl, val, x, y);
        default: return xab_fail(ctx, XAB_E_UNSUPPORTED, "col_block %d", pl->params.col_block);
    }
}

XAB_INSTANTIATE_LAUNCHER(launch_nnz)
XAB_INSTANTIATE_LAUNCHER(launch_bss)
XAB_INSTANTIATE_LAUNCHER(launch_sym_s3)
XAB_INSTANTIATE_LAUNCHER(launch_xcb)

}  // namespace xab
