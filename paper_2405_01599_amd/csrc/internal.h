// Internal definitions of the xab library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/xab.h"

// ------------------------------------------------------------------ context
struct xab_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *user = nullptr;
    int policy = XAB_TIME;
    char err[512] = {0};
    // device scratch owned by the context (grown on demand)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    std::unordered_map<const void *, size_t> live;  // bytes of every block from xab_dalloc not yet freed
    int *d_flag = nullptr;          // validation error flags
    // cost model (host copy; uploaded on use)
    std::vector<float> mlp;         // XAB_MLP_NPARAMS
    std::vector<float> fmean, fstd; // 12 each
    bool mlp_set = false;
    float *d_mlp = nullptr;         // device copy of mlp + mean + std
};

struct xab_matrix {
    xab_ctx *ctx = nullptr;
    int32_t n = 0, ncols = 0;
    int64_t nnz = 0;
    const int32_t *rowptr = nullptr;
    const int32_t *colind = nullptr;
    const double *val64 = nullptr;
    const float *val32 = nullptr;
    bool has64 = false, has32 = false; // value copies attached (pointers may be null when nnz = 0)
    uint32_t flags = 0;
    bool sym() const { return (flags & XAB_SYM_LOWER) != 0; }
    // cached statistics (computed on first feature request)
    bool have_stats = false;
    int64_t stats[9] = {0};
    double *diag64 = nullptr; // Jacobi diagonal (lazy, library-owned)
    float *diag32 = nullptr;
};

// Sliced ELLPACK copy of a CSR (SELL-C-sigma, C = 64): rows ordered longest
// first inside windows of sigma rows, chunks of 64 ordered rows stored
// column-major and padded to the chunk's longest row.
struct xab_sell {
    int64_t nch = 0, total = 0;  // chunks, padded entries
    int32_t sigma = 0;
    int32_t *perm = nullptr;     // original row of ordered row r
    int32_t *rlen = nullptr;     // length of ordered row r (nch * 64 slots, 0 past n)
    int32_t *clen = nullptr;     // chunk widths
    int64_t *cptr = nullptr;     // [nch + 2] chunk offsets, padded size, widest chunk
    int32_t *cols = nullptr;     // padded columns (padding: 0)
    double *val64 = nullptr;     // padded values (padding: 0)
    float *val32 = nullptr;
};

struct xab_plan {
    xab_ctx *ctx = nullptr;
    const xab_matrix *A = nullptr;
    xab_variant variant = XAB_NNZ;
    xab_params params{};
    int64_t P = 0;             // tiles / parts / workgroups
    // NNZ: b[P+1]; SYM_S3: b[P+1] tile row boundaries
    int32_t *b = nullptr;
    // BSS
    int32_t *row_lo = nullptr, *tile_row = nullptr, *carry_row = nullptr;
    void *carry_val = nullptr, *tail_val = nullptr; // acc-type workspaces [P]
    int32_t *tail_row = nullptr;
    // SYM_S3 touch map
    int64_t nblk = 0, ntouch = 0;
    int32_t *tm_ptr = nullptr, *tm_tile = nullptr, *tile_ptr = nullptr, *tile_blk = nullptr, *tile_slot = nullptr;
    int32_t *tile_minblk = nullptr;
    void *partial = nullptr;   // ntouch * col_block acc-type values
    size_t partial_elem = 0;   // bytes per element allocated (4 or 8)
    int32_t s3_own_cap = 0;    // most rows of a tile
    int32_t s3_ext_cap = 0;    // most touched blocks of a tile times col_block
    int32_t s3_lut_cap = 0;    // widest span of touched block ids of a tile
    int32_t s3_walk = 0;       // 0: walk over the CSR entry stream, 1: sliced walk (lane = row)
    // stream walk: copy of colind, bit 31 on the first entry of every non-empty
    // row, bit 30 on an entry added after its chunk's slots
    int32_t *s3_ci = nullptr;
    uint8_t *s3_dense = nullptr; // per tile: 1 when none of its rows is empty (the flagged walk applies)
    // sliced walk: each tile's rows in chunks of 64 (the last one partial),
    // every chunk stored column-major (stride = its row count), padded to
    // its longest row; columns carry bit 30 like the stream walk's
    int64_t s3_nch = 0;          // chunks
    int64_t s3_padded = 0;       // padded entries
    int32_t *s3_ch0 = nullptr;   // [P + 1] first chunk of each tile
    int32_t *s3_cw = nullptr;    // [nch] chunk widths
    int64_t *s3_coff = nullptr;  // [nch + 1] chunk offsets (the last = padded size)
    int32_t *s3_cols = nullptr;  // padded columns (padding: -1)
    double *s3_v64 = nullptr;    // padded values (padding: 0)
    float *s3_v32 = nullptr;
    // XCB: column-blocked copy of the matrix, one CSR per column block
    static constexpr int kXcb = 8;
    int32_t *xcb_rowptr = nullptr;      // kXcb * (n + 1), each relative to its block's first entry
    uint8_t *xcb_mask = nullptr;        // n: bit k set when row i has entries in block k
    int64_t xcb_m[kXcb] = {0};          // non-empty rows per block (the block's compressed rows)
    int32_t *xcb_colind = nullptr;      // nnz, the blocks concatenated; bit 31 flags a compressed row's first entry
    double *xcb_val64 = nullptr;        // copies of the values in the same order
    float *xcb_val32 = nullptr;
    int64_t xcb_base[kXcb + 1] = {0};   // block k holds entries [base[k], base[k+1])
    int64_t xcb_P[kXcb] = {0};          // segmented-scan tiles per block
    int64_t xcb_toff[kXcb + 1] = {0};   // tile offsets of the blocks in the descriptor arrays
    int32_t *xcb_row_lo = nullptr, *xcb_carry_row = nullptr, *xcb_tail_row = nullptr, *xcb_tile_row = nullptr;
    void *xcb_carry_val = nullptr, *xcb_tail_val = nullptr;  // acc-type, per tile
    int64_t xcb_ybase[kXcb + 1] = {0};  // block k's partials: Y[ybase[k] .. ybase[k] + m_k)
    void *xcb_Y = nullptr;              // compressed partial products, acc-type, ybase[kXcb] slots
    int64_t xcb_G = 0;                  // row groups of 256 (the combine's workgroups)
    int32_t *xcb_gbase = nullptr;       // kXcb * (G + 1): compressed index of group g's first row in block k
    // column window of this plan's blocks (the whole matrix unless it is
    // one slice of a sliced plan) and, for a sliced plan, one plan per
    // slice plus the accumulation-type sum carried from slice to slice
    int32_t xcb_c0 = 0, xcb_c1 = 0;
    std::vector<xab_plan *> xcb_sub;
    void *xcb_ysum = nullptr;
    // FP32 values walked with fewer entries per lane than FP64 ones (when
    // the plan chose J from the size): their own lane-interleaved copy of
    // the columns and their own tiles; partials, mask and group offsets
    // are shared.  xcb_j32 = 0: the FP32 values use the FP64 walk.
    int32_t xcb_j32 = 0;
    int32_t *xcb_colind32 = nullptr;
    int64_t xcb_P32[kXcb] = {0};
    int64_t xcb_toff32[kXcb + 1] = {0};
    int32_t *xcb_row_lo32 = nullptr, *xcb_carry_row32 = nullptr, *xcb_tail_row32 = nullptr, *xcb_tile_row32 = nullptr;
    void *xcb_carry_val32 = nullptr, *xcb_tail_val32 = nullptr;
    // SELL: chunks of kSellC ordered rows, column-major, padded to the chunk's longest row
    static constexpr int kSellC = 64;
    static constexpr int kSellMaxRow = 4096;
    xab_sell sell;
    // BCSR: 4 x 4 blocks, 16 values row-major per block
    static constexpr int kBcsrB = 4;
    static constexpr int kBcsrMaxRow = 4096;  // entries of one block row (set-up sorts them in LDS)
    int64_t bcsr_nbr = 0, bcsr_nb = 0;
    int32_t *bcsr_brp = nullptr;   // [nbr + 1] block row pointers
    int32_t *bcsr_bci = nullptr;   // block columns, ascending within a block row
    int32_t *bcsr_mask = nullptr;  // bit (r % 4) * 4 + c % 4 for every stored position
    double *bcsr_val64 = nullptr;
    float *bcsr_val32 = nullptr;
};

struct xab_batch {
    xab_ctx *ctx = nullptr;
    int32_t nsys = 0;
    int64_t n = 0, nnz = 0;
    std::vector<int64_t> row_off, nnz_off;
    const int32_t *rowptr = nullptr, *colind = nullptr;
    const void *val = nullptr;
    xab_dtype vt = XAB_F64;
    // segmented-scan tiles of the concatenated matrix (kBatchJ entries per lane)
    int64_t P = 0;
    int32_t *row_lo = nullptr, *tile_row = nullptr, *carry_row = nullptr, *tail_row = nullptr;
    double *carry_val = nullptr, *tail_val = nullptr;
    int32_t *d_sys_of_row = nullptr; // system index of every row
    int64_t *d_row_off = nullptr;    // [nsys+1]
    // BiCGStab row segments: segment j covers rows of system d_seg_sys[j];
    // system k owns segments [d_seg_off[k], d_seg_off[k+1])
    int64_t nseg = 0;
    int32_t *d_seg_sys = nullptr, *d_seg_off = nullptr;
    void *diag = nullptr;            // Jacobi diagonal (value type; lazy, library-owned)
    xab_sell sell;                   // sliced ELLPACK copy (when within its limits): the SpMV of choice
};

// ------------------------------------------------------------------ helpers
int xab_fail(xab_ctx *ctx, int code, const char *fmt, ...);
void *xab_dalloc(xab_ctx *ctx, size_t bytes);
void xab_dfree(xab_ctx *ctx, void *p);
int xab_hip_check(xab_ctx *ctx, hipError_t e, const char *what);
// scratch: at least `bytes` of context-owned device memory (reused across calls)
void *xab_scratch(xab_ctx *ctx, size_t bytes);
// bytes of a live block from xab_dalloc (0 for NULL or unknown pointers)
size_t xab_dbytes(const xab_ctx *ctx, const void *p);

#define XAB_HIP(ctx, call)                                   \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return xab_hip_check(ctx, _e, #call); \
    } while (0)

#define XAB_LAUNCH_CHECK(ctx, what)                                        \
    do {                                                                   \
        hipError_t _e = hipGetLastError();                                 \
        if (_e != hipSuccess) return xab_hip_check(ctx, _e, what);         \
    } while (0)

// plan builders (plan.hip)
int xab_build_plan(xab_ctx *ctx, const xab_matrix *A, xab_variant v, const xab_params *p, xab_plan **out);
// SELL copy of a CSR (plan.hip): XAB_E_UNSUPPORTED when a row is longer
// than 4096 or the padded size exceeds 2 nnz + 64 * (longest row); the
// arrays are then freed.  Synchronous.
int xab_sell_build(xab_ctx *ctx, const int32_t *rowptr, const int32_t *colind, const double *v64, const float *v32,
                   bool has64, bool has32, int32_t n, int64_t nnz, int32_t sigma, xab_sell *out);
void xab_sell_free(xab_ctx *ctx, xab_sell *s);
// segmented-scan tile descriptors (row_lo, tile_row [P+1], carry_row [P]) of a
// CSR with T entries per tile, queued on `st`
void xab_launch_split_bss(hipStream_t st, const int32_t *rowptr, int32_t n, int64_t T, int64_t P, int32_t *row_lo,
                          int32_t *tile_row, int32_t *carry_row);

// the allocation-free SpMV's device buffer: its address on the context's
// device, looked up once per device (noalloc.hip; called by xab_init)
int xab_noalloc_setup(xab_ctx *ctx);

// SpMV dispatch (spmv.hip)
int xab_spmv_dispatch(xab_ctx *ctx, const xab_plan *plan, const void *x, xab_dtype xt, void *y, xab_dtype yt,
                      xab_dtype acc);

// statistics (features.hip)
int xab_matrix_stats(xab_ctx *ctx, xab_matrix *A);
void xab_stats_to_features(const int64_t *st, int sym, float *out);

// Jacobi diagonal (blas.hip)
int xab_matrix_diag(xab_ctx *ctx, xab_matrix *A);

// ------------------------------------------------------------------ device helpers
#ifdef __HIPCC__
namespace xab {

constexpr int kWave = 64;

// Number of XCDs of the MI355X: consecutive workgroup ids are dispatched
// round-robin over them.  xcd_remap turns a hardware block id into a
// logical tile index such that each XCD receives a contiguous range of
// tiles (its L2 then caches one window of x instead of the whole vector).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
    int64_t q = nblocks / kXcds, r = nblocks % kXcds;
    int64_t xcd = bid % kXcds, i = bid / kXcds;
    return xcd * q + (xcd < r ? xcd : r) + i;
}

template <class T>
__device__ __forceinline__ T ld_nt(const T *p) {
    return __builtin_nontemporal_load(p);
}

template <class T>
__device__ __forceinline__ T shfl_up(T v, int d) {
    return __shfl_up(v, d, kWave);
}
template <class T>
__device__ __forceinline__ T shfl_xor(T v, int m, int w = kWave) {
    return __shfl_xor(v, m, w);
}

// Segmented-sum scan element: `f` = a segment (row) starts in this span,
// `v` = sum since the last start (or of the whole span), `r` = row of that
// last start.  combine(a, b) = the state after a followed by b.
template <class AT>
struct Seg {
    int f;
    AT v;
    int r;
};
template <class AT>
__device__ __forceinline__ Seg<AT> seg_combine(const Seg<AT> &a, const Seg<AT> &b) {
    Seg<AT> o;
    o.f = a.f | b.f;
    o.v = b.f ? b.v : a.v + b.v;
    o.r = b.f ? b.r : a.r;
    return o;
}

// Cross-lane moves with the data-parallel primitives (DPP) of the GFX9 ISA:
// a VALU move that reads another lane of the wave, no LDS round trip.
// Lanes whose source is disabled (outside the 16-lane row for row_shr, or
// in rows left out of ROW_MASK for the row broadcasts) read 0: the all-zero
// state is the identity of every scan combine that uses these moves.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, dpp_move<CTRL, ROW_MASK>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_move<CTRL, ROW_MASK>((int)(unsigned)(b & 0xffffffffull));
    const unsigned hi = (unsigned)dpp_move<CTRL, ROW_MASK>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Inclusive scan across the 64 lanes of a wave for an associative combine
// whose identity is the all-zero state: Kogge-Stone inside each 16-lane
// row (shifts 1, 2, 4, 8), then row 0's total into row 1 and row 2's into
// row 3 (broadcast of lane 15), then the first half's total into rows 2
// and 3 (broadcast of lane 31).  Step(u, s) must return combine(u, s) with
// u the DPP-moved copy of s.
template <class S, class Step>
__device__ __forceinline__ S wave_scan_dpp(S s, Step step) {
    s = step.template apply<kDppRowShr1, 0xf>(s);
    s = step.template apply<kDppRowShr2, 0xf>(s);
    s = step.template apply<kDppRowShr4, 0xf>(s);
    s = step.template apply<kDppRowShr8, 0xf>(s);
    s = step.template apply<kDppRowBcast15, 0xa>(s);
    s = step.template apply<kDppRowBcast31, 0xc>(s);
    return s;
}

struct SegStep {
    template <int CTRL, int RM, class AT>
    __device__ __forceinline__ Seg<AT> apply(const Seg<AT> &s) const {
        const Seg<AT> u{dpp_move<CTRL, RM>(s.f), dpp_move<CTRL, RM>(s.v), dpp_move<CTRL, RM>(s.r)};
        return seg_combine(u, s);
    }
};

// Inclusive segmented scan across the 64 lanes of a wave.
template <class AT>
__device__ __forceinline__ Seg<AT> wave_seg_scan(Seg<AT> s, int) {
    return wave_scan_dpp(s, SegStep{});
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) v += shfl_xor(v, m);
    return v;
}

}  // namespace xab
#endif
