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
constexpr int kSymJ = sym::kChunkJ;  // entries per lane per chunk (symmetric)

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
                                                     int lut_cap, const int32_t *__restrict__ ci_f,
                                                     const uint8_t *__restrict__ dense) {
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

    if (dense[p]) {
        // every row of the tile is non-empty: walk the flagged copy of the
        // columns (rows found by counting heads, no row pointers), with the
        // next chunk's loads and gathers in flight while one is scanned
        struct LocalSink {
            Sink &s;
            int32_t r0;
            __device__ void row_done(int32_t l, AT v) { s.row_done(r0 + l, v); }
            __device__ void entry(int32_t l, int32_t j, VT v) { s.entry(r0 + l, j, v); }
        } ls{sink, r0};
        CSeg<AT> *cwave = (CSeg<AT> *)wave_tot;
        const int64_t A0 = s - (s % CH);
        Run<kSymJ, VT, XT> R0, R1;
        run_load<kNT, kSymJ>(R0, A0, s, e < A0 + CH ? e : A0 + CH, ci_f, val);
        run_gather_flagged(R0, x);
        if (A0 + CH < e) run_load<kNT, kSymJ>(R1, A0 + CH, A0 + CH, e < A0 + 2 * CH ? e : A0 + 2 * CH, ci_f, val);
        CSeg<AT> st{0, AT(0)};
        for (int64_t A = A0;; A += CH) {
            const bool last = A + CH >= e;
            if (!last) run_gather_flagged(R1, x);
            Run<kSymJ, VT, XT> R2;
            if (A + 2 * CH < e)
                run_load<kNT, kSymJ>(R2, A + 2 * CH, A + 2 * CH, e < A + 3 * CH ? e : A + 3 * CH, ci_f, val);
            st = flag_chunk<kNT, kSymJ, VT, XT, AT>(R0, st, cwave, ls);
            if (last) break;
            R0 = R1;
            R1 = R2;
        }
        if (tid == 0 && st.c > 0) atomicAdd(&own[st.c - 1], st.v);
    } else {
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
    }
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
    const size_t lds = sym_lds_bytes<AT>(pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap);
    if (lds > (size_t)sym::kLdsCap)
        return xab_fail(ctx, XAB_E_UNSUPPORTED, "symmetric tile needs %zu bytes of LDS", lds);
    hipLaunchKernelGGL((k_spmv_sym_s3<VT, XT, YT, AT, C>), dim3((unsigned)pl->P), dim3(kNT), lds, ctx->stream,
                       A->rowptr, A->colind, val, x, y, pl->b, pl->P, pl->tile_ptr, pl->tile_blk, pl->tile_slot,
                       pl->tile_minblk, (AT *)pl->partial, pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap,
                       pl->s3_ci, pl->s3_dense);
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
