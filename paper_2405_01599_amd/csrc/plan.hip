// Plan setup: the per-implementation data structures built before the
// run-time judge (the setup functions of the paper's Table 1).  All passes
// over the matrix run on the device; only the small list of
// (tile, column block) pairs of the symmetric touch map is ordered on the
// host.
#include <algorithm>
#include <climits>
#include <cstring>

#include "internal.h"
#include "sym_layout.h"
#include <type_traits>

namespace {

// smallest r in [0, n] with rowptr[r] >= target
__device__ __forceinline__ int32_t lower_bound_rp(const int32_t *rowptr, int32_t n, int64_t target) {
    int32_t lo = 0, hi = n + 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (rowptr[mid] >= target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// largest r in [0, n] with rowptr[r] <= target
__device__ __forceinline__ int32_t last_le_rp(const int32_t *rowptr, int32_t n, int64_t target) {
    int32_t lo = 0, hi = n + 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (rowptr[mid] <= target) lo = mid + 1;
        else hi = mid;
    }
    return lo - 1;
}

// nnz-based split: b[p] = lower_bound(floor(p * nnz / P)), b[0] = 0, b[P] = n
__global__ void k_split_nnz(const int32_t *rowptr, int32_t n, int64_t nnz, int64_t P, int32_t *b) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    int32_t v;
    if (p == 0) v = 0;
    else if (p == P) v = n;
    else v = lower_bound_rp(rowptr, n, (p * nnz) / P);
    b[p] = v;
}

// segmented-scan tiles of T entries: first row starting in the tile, the
// row holding the tile's first entry, and the carried-in row (or -1)
__global__ void k_split_bss(const int32_t *rowptr, int32_t n, int64_t T, int64_t P, int32_t *row_lo,
                            int32_t *tile_row, int32_t *carry_row) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > P) return;
    if (t == P) {
        row_lo[P] = n;
        tile_row[P] = n;
        return;
    }
    int64_t e = t * T;
    int32_t lo = lower_bound_rp(rowptr, n, e);
    int32_t tr = last_le_rp(rowptr, n, e);
    if (tr > n - 1) tr = n - 1;
    if (tr < 0) tr = 0;
    row_lo[t] = lo;
    tile_row[t] = tr;
    carry_row[t] = (n > 0 && rowptr[tr] < e) ? tr : -1;
}

// Symmetric tiles in whole 256-row groups (four 64-row chunks, one round
// of the sliced walk's four waves): with Rmax >= 256 the inner boundaries
// of the nnz split move to the nearest multiple of 256 rows (at most n)
__global__ void k_sym_round(int32_t *b0, int64_t P0, int32_t n, int32_t Rmax) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < 1 || p >= P0 || Rmax < 256) return;
    const int64_t r = (((int64_t)b0[p] + 128) / 256) * 256;
    b0[p] = (int32_t)(r < n ? r : n);
}

// step 1: pieces per part.  An empty part is dropped (unless it is the
// only one); with Rmax >= 256 a part of R rows is cut into ceil(u / g)
// pieces of whole groups (u = ceil(R / 256) groups, at most g = Rmax / 256
// per piece), else into ceil(R / Rmax) pieces
__global__ void k_sym_pieces(const int32_t *b0, int64_t P0, int32_t Rmax, int32_t *cnt) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P0) return;
    const int64_t R = b0[p + 1] - b0[p];
    int64_t k;
    if (R == 0 && P0 > 1) k = 0;
    else if (Rmax >= 256) k = (((R + 255) / 256) + Rmax / 256 - 1) / (Rmax / 256);
    else k = (R + Rmax - 1) / Rmax;
    cnt[p] = (int32_t)(R == 0 && P0 > 1 ? 0 : (k < 1 ? 1 : k));
}

// step 2: piece i of part p starts at b0[p] + 256 floor(i u / k) (whole
// groups) or b0[p] + floor(i R / k)
__global__ void k_sym_fill(const int32_t *b0, const int32_t *cnt, const int32_t *off, int64_t P0, int32_t n,
                           int32_t Rmax, int32_t *b) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P0) return;
    if (p == P0) {
        b[off[P0]] = n;
        return;
    }
    const int64_t R = b0[p + 1] - b0[p];
    const int32_t k = cnt[p];
    const int64_t u = (R + 255) / 256;
    for (int32_t i = 0; i < k; ++i)
        b[off[p] + i] = (int32_t)(b0[p] + (Rmax >= 256 ? 256 * ((i * u) / k) : (i * R) / k));
}

// Exclusive scan of a small int array in one workgroup: out[0..m] (out[m] = total).
__global__ void k_scan_small(const int32_t *in, int64_t m, int32_t *out) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < m; base += 1024) {
        int64_t i = base + tid;
        int64_t v = i < m ? in[i] : 0;
        part[tid] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t u = tid >= d ? part[tid - d] : 0;
            __syncthreads();
            part[tid] += u;
            __syncthreads();
        }
        if (i < m) out[i] = (int32_t)(carry + part[tid] - v);
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
    if (tid == 0) out[m] = (int32_t)carry;
}

constexpr int kSpanBad = 1, kCountBad = 2;

// step 3: per tile, the set of column blocks below the tile's first row that
// its transposed entries land in, as a bitmap over [minblk, minblk + span)
__global__ __launch_bounds__(256) void k_sym_touch(const int32_t *rowptr, const int32_t *colind,
                                                   const int32_t *b, int64_t P, int32_t C, int32_t bmax,
                                                   int32_t *tile_minblk, int32_t *cnt, uint32_t *bitmap,
                                                   int *flag) {
    __shared__ int32_t red[256];
    __shared__ uint32_t bits[xab::sym::kLutWords];
    int64_t p = blockIdx.x;
    int tid = threadIdx.x;
    int32_t r0 = b[p], r1 = b[p + 1];
    int64_t s = rowptr[r0], e = rowptr[r1];
    int32_t mn = INT_MAX;
    for (int64_t k = s + tid; k < e; k += 256) {
        int32_t j = colind[k];
        if (j < r0 && j < mn) mn = j;
    }
    red[tid] = mn;
    if (tid < xab::sym::kLutWords) bits[tid] = 0u;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (tid < d) red[tid] = min(red[tid], red[tid + d]);
        __syncthreads();
    }
    int32_t minj = red[0];
    int32_t minblk = (minj == INT_MAX) ? 0 : minj / C;
    int bad = 0;
    if (minj != INT_MAX) {
        for (int64_t k = s + tid; k < e; k += 256) {
            int32_t j = colind[k];
            if (j < r0) {
                int32_t d = j / C - minblk;
                if (d >= xab::sym::kLutMax) bad |= kSpanBad;
                else atomicOr(&bits[d >> 5], 1u << (d & 31));
            }
        }
    }
    __syncthreads();
    int c = 0;
    if (tid < xab::sym::kLutWords) c = __popc(bits[tid]);
    red[tid] = c;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (tid < d) red[tid] += red[tid + d];
        __syncthreads();
    }
    if (tid == 0) {
        cnt[p] = red[0];
        tile_minblk[p] = minblk;
        if (red[0] > bmax) bad |= kCountBad;
    }
    if (tid < xab::sym::kLutWords) bitmap[p * xab::sym::kLutWords + tid] = bits[tid];
    if (bad) atomicOr(flag, bad);
}

// step 4: the tile's blocks in ascending order
__global__ void k_sym_blocks(const uint32_t *bitmap, const int32_t *tile_minblk, const int32_t *tile_ptr,
                             int32_t *tile_blk) {
    __shared__ int32_t pre[xab::sym::kLutWords];
    int64_t p = blockIdx.x;
    int w = threadIdx.x;
    uint32_t word = bitmap[p * xab::sym::kLutWords + w];
    pre[w] = __popc(word);
    __syncthreads();
    if (w == 0) {
        int32_t acc = 0;
        for (int i = 0; i < xab::sym::kLutWords; ++i) {
            int32_t v = pre[i];
            pre[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int32_t pos = tile_ptr[p] + pre[w];
    int32_t base = tile_minblk[p] + w * 32;
    while (word) {
        int bit = __ffs(word) - 1;
        tile_blk[pos++] = base + bit;
        word &= word - 1;
    }
}

__global__ void k_fill_flag(int *f) {
    if (threadIdx.x == 0) *f = 0;
}

// ---- column-blocked copy (XCB): block of a column, counts, scan, scatter
struct ColBlocks {
    int32_t cb[xab_plan::kXcb + 1];  // block k = columns [cb[k], cb[k+1])
};

// the column block of col, -1 outside the window [cb[0], cb[kXcb])
__device__ __forceinline__ int col_block_of(const ColBlocks &c, int32_t col) {
    if (col < c.cb[0] || col >= c.cb[xab_plan::kXcb]) return -1;
    int k = 0;
#pragma unroll
    for (int q = 1; q < xab_plan::kXcb; ++q) k += col >= c.cb[q];
    return k;
}

// cnt[k * n + i] = entries of row i in column block k
__global__ void k_xcb_count(const int32_t *rowptr, const int32_t *colind, int32_t n, ColBlocks c, int32_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t m[xab_plan::kXcb] = {0};
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        int k = col_block_of(c, colind[e]);
#pragma unroll
        for (int q = 0; q < xab_plan::kXcb; ++q) m[q] += (q == k);
    }
#pragma unroll
    for (int q = 0; q < xab_plan::kXcb; ++q) cnt[(int64_t)q * n + i] = m[q];
}

// Exclusive scan of in[0..m) into out[0..m] (out[m] = total) in three
// steps: per-workgroup sums of 2048 elements, a scan of those sums, and a
// per-workgroup rescan with its offset.
constexpr int kScanItems = 8, kScanTile = 256 * kScanItems;

__global__ void k_scan_tile_sums(const int32_t *in, int64_t m, int32_t *sums) {
    __shared__ int32_t red[256];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t a = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < m) a += in[base + q];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void k_scan_tile_apply(const int32_t *in, int64_t m, const int32_t *offs, int32_t *out) {
    __shared__ int32_t part[256];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems], a = 0;
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < m ? in[base + q] : 0;
        a += v[q];
    }
    part[threadIdx.x] = a;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        int32_t u = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += u;
        __syncthreads();
    }
    int32_t run = offs[blockIdx.x] + part[threadIdx.x] - a;
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < m) out[base + q] = run;
        run += v[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[m] = offs[gridDim.x];  // the total
}

// mask[i] bit k = row i has entries in block k; flag_k[i] = that bit for one block
__global__ void k_xcb_mask(const int32_t *cnt, int32_t n, uint8_t *mask) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t m = 0;
    for (int k = 0; k < xab_plan::kXcb; ++k) m |= (cnt[(int64_t)k * n + i] > 0 ? 1u : 0u) << k;
    mask[i] = (uint8_t)m;
}

__global__ void k_nonzero_flags(const int32_t *cnt, int32_t n, int32_t *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = cnt[i] > 0;
}

// a block's CSR restricted to its non-empty rows: crp[j] = start of the
// j-th such row, crp[m] = the block's size
__global__ void k_xcb_compress(const int32_t *flag, const int32_t *pos, const int32_t *rp_full, int32_t n,
                               int32_t *crp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        crp[pos[n]] = rp_full[n];
        return;
    }
    if (flag[i]) crp[pos[i]] = rp_full[i];
}

// bit 31 on the first entry of each of the block's m non-empty rows
__global__ void k_xcb_flag_heads(const int32_t *crp, int32_t m, int32_t *ci) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int32_t e = crp[r];
    ci[e] = (int32_t)((uint32_t)ci[e] | 0x80000000u);
}

// bit 31 on the first entry of every non-empty row of a CSR (in place on a copy)
__global__ void k_flag_row_heads(const int32_t *rowptr, int32_t n, int32_t *ci) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t e0 = rowptr[r];
    if (rowptr[r + 1] > e0) ci[e0] = (int32_t)((uint32_t)ci[e0] | 0x80000000u);
}

// bit 30 of the symmetric column copy: entry q of tile p is added after
// its chunk's slots when an entry of the same tile, the same chunk of
// sym::kChunk entries and the same slot (q - J, q - 2J, ... down to the
// chunk's or the tile's start) has the same column
__global__ __launch_bounds__(256) void k_sym_defer(const int32_t *rowptr, const int32_t *colind, const int32_t *b,
                                                   int32_t *ci) {
    constexpr int J = xab::sym::kChunkJ, CH = xab::sym::kChunk;
    const int64_t p = blockIdx.x;
    const int64_t s = rowptr[b[p]], e = rowptr[b[p + 1]];
    for (int64_t q = s + threadIdx.x; q < e; q += 256) {
        const int32_t j = colind[q];
        const int64_t c0 = q - q % CH, lo = c0 > s ? c0 : s;
        bool d = false;
        for (int64_t u = q - J; u >= lo && !d; u -= J) d = colind[u] == j;
        if (d) ci[q] = (int32_t)((uint32_t)ci[q] | xab::sym::kDeferBit);
    }
}

// sliced symmetric walk, step 1: chunks of 64 rows per tile (the last
// one partial)
__global__ void k_sym_nch(const int32_t *b, int64_t P, int32_t *cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) cnt[p] = (b[p + 1] - b[p] + xab::sym::kLanes - 1) / xab::sym::kLanes;
}

// step 2 (one wave per tile): each chunk's width (its longest row) and
// stored size (width x rows); the widest chunk goes to *widest
__global__ __launch_bounds__(64) void k_sym_widths(const int32_t *rowptr, const int32_t *b, const int32_t *ch0,
                                                   int32_t *cw, int64_t *csz, int *widest) {
    const int64_t p = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t r0 = b[p], r1 = b[p + 1], g0 = ch0[p];
    int32_t most = 0;
    for (int32_t g = g0; g < ch0[p + 1]; ++g) {
        const int32_t rc = r0 + xab::sym::kLanes * (g - g0);
        const int32_t i = rc + lane;
        int32_t w = i < r1 ? rowptr[i + 1] - rowptr[i] : 0;
        for (int m = 32; m > 0; m >>= 1) w = max(w, __shfl_xor(w, m, 64));
        if (lane == 0) {
            cw[g] = w;
            csz[g] = (int64_t)w * min(xab::sym::kLanes, r1 - rc);
        }
        most = max(most, w);
    }
    if (lane == 0) atomicMax(widest, most);
}

// exclusive scan of int64 values in one workgroup: out[0..m] (out[m] = total)
__global__ void k_scan_i64(const int64_t *in, int64_t m, int64_t *out) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < m; base += 1024) {
        const int64_t i = base + t;
        const int64_t v = i < m ? in[i] : 0;
        part[t] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int64_t u = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        if (i < m) out[i] = carry + part[t] - v;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
    if (t == 0) out[m] = carry;
}

// step 3 (one wave per tile): the padded column-major copy.  Entry k of
// the chunk's lane l (row r0 + 64 c + l) sits at coff[g] + k * rows + l;
// padding has column -1 and value 0.  Bit 30: a lower lane of the same
// chunk has the same column in slot k.
__global__ __launch_bounds__(64) void k_sym_slice_fill(const int32_t *rowptr, const int32_t *colind,
                                                       const double *v64, const float *v32, const int32_t *b,
                                                       const int32_t *ch0, const int32_t *cw, const int64_t *coff,
                                                       int32_t *cols, double *o64, float *o32) {
    __shared__ int32_t slot[64];
    const int64_t p = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t r0 = b[p], r1 = b[p + 1], g0 = ch0[p];
    for (int32_t g = g0; g < ch0[p + 1]; ++g) {
        const int32_t rc = r0 + xab::sym::kLanes * (g - g0);
        const int32_t i = rc + lane, nr = min(xab::sym::kLanes, r1 - rc);
        const bool on = lane < nr;
        const int32_t s = on ? rowptr[i] : 0, len = on ? rowptr[i + 1] - s : 0;
        const int32_t w = cw[g];
        const int64_t o = coff[g];
        for (int32_t k = 0; k < w; ++k) {
            const int32_t c = k < len ? colind[s + k] : -1;
            slot[lane] = c;
            __syncthreads();
            bool later = false;
            if (c >= 0)
                for (int l = 0; l < lane; ++l) later |= slot[l] == c;
            __syncthreads();
            if (on) {
                const int64_t q = o + (int64_t)k * nr + lane;
                if (cols) cols[q] = later ? (int32_t)((uint32_t)c | xab::sym::kDeferBit) : c;
                if (o64) o64[q] = k < len ? v64[s + k] : 0.0;
                if (o32) o32[q] = k < len ? v32[s + k] : 0.0f;
            }
        }
    }
}

// The column-blocked copy's full tiles are stored in 16-byte groups
// interleaved over the lanes: with G = min(J, 16 / element size) entries
// per group, entry q of lane t of a tile of T = 256 J entries (block
// position tile T + t J + q) moves to tile T + (q / G) 256 G + t G + q % G,
// so each wide load of the SpMV reads 256 consecutive groups (G = J keeps
// the plain order); a block's last, partial tile keeps its order
template <class T>
__global__ void k_xcb_interleave(const T *in, T *out, int64_t nnz, int32_t J) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    const int64_t TT = 256 * (int64_t)J;
    const int64_t G = std::min<int64_t>(J, 16 / (int64_t)sizeof(T));
    const int64_t tile = i / TT;
    int64_t dst = i;
    if (tile < nnz / TT) {
        const int64_t r = i - tile * TT, t = r / J, q = r % J;
        dst = tile * TT + (q / G) * 256 * G + t * G + q % G;
    }
    out[dst] = in[i];
}

// dense[p] = 1 when every row of tile p (rows [b[p], b[p+1])) has an entry
__global__ void k_tile_dense(const int32_t *rowptr, const int32_t *b, int64_t P, uint8_t *dense) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint8_t d = 1;
    for (int32_t r = b[p]; r < b[p + 1] && d; ++r) d = rowptr[r + 1] > rowptr[r];
    dense[p] = d;
}

// cnt[k * G + g] = rows of group g (256 rows) with entries in block k
__global__ void k_xcb_group_counts(const uint8_t *mask, int32_t n, int64_t G, int32_t *cnt) {
    __shared__ int32_t c[xab_plan::kXcb];
    if (threadIdx.x < xab_plan::kXcb) c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t m = i < n ? mask[i] : 0u;
    for (int k = 0; k < xab_plan::kXcb; ++k)
        if ((m >> k) & 1u) atomicAdd(&c[k], 1);
    __syncthreads();
    if (threadIdx.x < xab_plan::kXcb) cnt[(int64_t)threadIdx.x * G + blockIdx.x] = c[threadIdx.x];
}

// stable scatter of every row's entries into its column block's CSR
__global__ void k_xcb_scatter(const int32_t *rowptr, const int32_t *colind, const double *v64, const float *v32,
                              int32_t n, ColBlocks c, const int32_t *rp, const int64_t *base, int32_t *ci_out,
                              double *v64_out, float *v32_out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t pos[xab_plan::kXcb];
#pragma unroll
    for (int q = 0; q < xab_plan::kXcb; ++q) pos[q] = base[q] + rp[(int64_t)q * (n + 1) + i];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        int32_t col = colind[e];
        int k = col_block_of(c, col);
        if (k < 0) continue;
        int64_t p = 0;
#pragma unroll
        for (int q = 0; q < xab_plan::kXcb; ++q)
            if (q == k) p = pos[q]++;
        if (ci_out) ci_out[p] = col;
        if (v64) v64_out[p] = v64[e];
        if (v32) v32_out[p] = v32[e];
    }
}

template <class T>
__global__ void k_fill_zero(T *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = T(0);
}

__global__ void k_zero_i32(int32_t *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0;
}

// ---- SELL-C-sigma: order rows inside each window, chunk widths, padded copy
// One workgroup (blockDim = the window rounded up to a power of two, at
// most 1024) per window: bitonic sort of (longest first, then lower row)
// keys in LDS.
__global__ void k_sell_sort(const int32_t *rowptr, int32_t n, int32_t sigma, int32_t *perm, int32_t *rlen) {
    __shared__ unsigned long long key[1024];
    const int P2 = blockDim.x;
    const int64_t w0 = (int64_t)blockIdx.x * sigma;
    const int t = threadIdx.x;
    const int64_t r = w0 + t;
    unsigned long long k = ~0ull;
    if (t < sigma && r < n) {
        const uint32_t len = (uint32_t)(rowptr[r + 1] - rowptr[r]);
        k = ((unsigned long long)(0x7fffffffu - len) << 32) | (unsigned long long)r;
    }
    key[t] = k;
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int partner = t ^ stride;
            if (partner > t) {
                const bool up = (t & size) == 0;
                const unsigned long long a = key[t], b = key[partner];
                if ((a > b) == up) {
                    key[t] = b;
                    key[partner] = a;
                }
            }
            __syncthreads();
        }
    }
    if (t < sigma && r < n) {
        const unsigned long long q = key[t];
        perm[r] = (int32_t)(q & 0xffffffffull);
        rlen[r] = (int32_t)(0x7fffffffu - (uint32_t)(q >> 32));
    }
}

// chunk widths: the first ordered row of a chunk is its longest (chunks lie
// inside windows); lanes past n count as empty rows
__global__ void k_sell_widths(const int32_t *rlen, int32_t n, int64_t nch, int32_t *clen) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nch) clen[c] = rlen[c * xab_plan::kSellC];
}

// cptr[c] = C * sum of widths before chunk c (int64), cptr[nch] = padded
// size, cptr[nch + 1] = the widest chunk (one workgroup)
__global__ void k_sell_scan(const int32_t *clen, int64_t nch, int64_t *cptr) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry, widest;
    const int t = threadIdx.x;
    if (t == 0) {
        carry = 0;
        widest = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < nch; base += 1024) {
        const int64_t i = base + t;
        const int64_t v = i < nch ? (int64_t)clen[i] * xab_plan::kSellC : 0;
        part[t] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int64_t u = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        if (i < nch) {
            cptr[i] = carry + part[t] - v;
            if (clen[i] > widest) atomicMax((unsigned long long *)&widest, (unsigned long long)clen[i]);
        }
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
    if (t == 0) {
        cptr[nch] = carry;
        cptr[nch + 1] = widest;
    }
}

// ------------------------------------------------------------------ BCSR
// One workgroup per block row R: the block columns c / 4 of the entries of
// rows 4R .. 4R+3 are loaded into LDS and sorted (bitonic, padded with
// INT_MAX to a power of two).  Returns the entry count, or -1 when it is
// above kBcsrMaxRow (nothing loaded).
constexpr int kBcsrNT = 256;

__device__ int bcsr_sorted_cols(const int32_t *rowptr, const int32_t *colind, int32_t n, int64_t R, int32_t *key) {
    constexpr int B = xab_plan::kBcsrB;
    const int64_t r0 = R * B, r1 = r0 + B < n ? r0 + B : n;
    const int32_t k0 = rowptr[r0];
    const int L = rowptr[r1] - k0;
    if (L > xab_plan::kBcsrMaxRow) return -1;
    int P2 = 1;
    while (P2 < L) P2 <<= 1;
    for (int i = threadIdx.x; i < P2; i += kBcsrNT) key[i] = i < L ? colind[k0 + i] / B : INT32_MAX;
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P2; i += kBcsrNT) {
                const int partner = i ^ stride;
                if (partner > i) {
                    const bool up = (i & size) == 0;
                    const int32_t a = key[i], b = key[partner];
                    if ((a > b) == up) {
                        key[i] = b;
                        key[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    return L;
}

// cnt[R] = distinct block columns of block row R; *bad = 1 when a block row is too long
__global__ __launch_bounds__(kBcsrNT) void k_bcsr_count(const int32_t *rowptr, const int32_t *colind, int32_t n,
                                                        int32_t *cnt, int *bad) {
    __shared__ int32_t key[xab_plan::kBcsrMaxRow];
    __shared__ int32_t red[kBcsrNT];
    const int64_t R = blockIdx.x;
    const int L = bcsr_sorted_cols(rowptr, colind, n, R, key);
    if (L < 0) {
        if (threadIdx.x == 0) {
            cnt[R] = 0;
            atomicOr(bad, 1);
        }
        return;
    }
    int c = 0;
    for (int i = threadIdx.x; i < L; i += kBcsrNT) c += (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int d = kBcsrNT / 2; d > 0; d >>= 1) {
        if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[R] = red[0];
}

// block columns of block row R at bci[brp[R] ..], then every entry added to
// its position (values and masks zeroed beforehand; duplicates summed)
__global__ __launch_bounds__(kBcsrNT) void k_bcsr_fill(const int32_t *rowptr, const int32_t *colind, const double *v64,
                                                       const float *v32, int32_t n, const int32_t *brp, int32_t *bci,
                                                       int32_t *mask, double *b64, float *b32) {
    constexpr int B = xab_plan::kBcsrB;
    __shared__ int32_t key[xab_plan::kBcsrMaxRow];
    __shared__ int32_t uniq[xab_plan::kBcsrMaxRow];
    __shared__ int32_t part[kBcsrNT];
    const int64_t R = blockIdx.x;
    const int L = bcsr_sorted_cols(rowptr, colind, n, R, key);
    if (L <= 0) return;
    // compaction of the distinct values: contiguous slices per thread, then a block scan
    const int per = (L + kBcsrNT - 1) / kBcsrNT;
    const int i0 = threadIdx.x * per, i1 = i0 + per < L ? i0 + per : L;
    int c = 0;
    for (int i = i0; i < i1; ++i) c += (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int d = 1; d < kBcsrNT; d <<= 1) {
        const int32_t u = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += u;
        __syncthreads();
    }
    int o = part[threadIdx.x] - c;
    const int U = part[kBcsrNT - 1];
    const int32_t base = brp[R];
    for (int i = i0; i < i1; ++i)
        if (i == 0 || key[i] != key[i - 1]) {
            uniq[o] = key[i];
            bci[base + o] = key[i];
            ++o;
        }
    __syncthreads();
    const int64_t r0 = R * B, r1 = r0 + B < n ? r0 + B : n;
    for (int64_t r = r0; r < r1; ++r)
        for (int32_t k = rowptr[r] + threadIdx.x; k < rowptr[r + 1]; k += kBcsrNT) {
            const int32_t col = colind[k], cb = col / B;
            int lo = 0, hi = U;  // first position with uniq[pos] >= cb
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (uniq[mid] < cb) lo = mid + 1;
                else hi = mid;
            }
            const int64_t blk = base + lo;
            const int e = (int)(r - r0) * B + col % B;
            atomicOr(&mask[blk], 1 << e);
            if (b64) atomicAdd(&b64[blk * B * B + e], v64[k]);
            if (b32) atomicAdd(&b32[blk * B * B + e], v32[k]);
        }
}

// one lane per ordered row slot (nch * C of them): copy its row into the
// chunk's columns, zeros past the row's end
__global__ void k_sell_fill(const int32_t *rowptr, const int32_t *colind, const double *v64, const float *v32,
                            int32_t n, int64_t nch, const int32_t *perm, const int32_t *rlen, const int64_t *cptr,
                            const int32_t *clen, int32_t *cols, double *o64, float *o32) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nch * xab_plan::kSellC) return;
    const int64_t c = r / xab_plan::kSellC, l = r % xab_plan::kSellC;
    const int32_t w = clen[c];
    const int32_t len = r < n ? rlen[r] : 0;
    const int64_t src = r < n ? rowptr[perm[r]] : 0;
    for (int32_t k = 0; k < w; ++k) {
        const int64_t dst = cptr[c] + (int64_t)k * xab_plan::kSellC + l;
        const bool live = k < len;
        if (cols) cols[dst] = live ? colind[src + k] : 0;
        if (o64) o64[dst] = live ? v64[src + k] : 0.0;
        if (o32) o32[dst] = live ? v32[src + k] : 0.0f;
    }
}

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

static void free_plan_arrays(xab_ctx *ctx, xab_plan *pl) {
    for (xab_plan *q : pl->xcb_sub) xab_plan_destroy(q);
    pl->xcb_sub.clear();
    xab_dfree(ctx, pl->xcb_ysum);
    pl->xcb_ysum = nullptr;
    xab_dfree(ctx, pl->b);
    xab_dfree(ctx, pl->row_lo);
    xab_dfree(ctx, pl->tile_row);
    xab_dfree(ctx, pl->carry_row);
    xab_dfree(ctx, pl->carry_val);
    xab_dfree(ctx, pl->tail_val);
    xab_dfree(ctx, pl->tail_row);
    xab_dfree(ctx, pl->tm_ptr);
    xab_dfree(ctx, pl->tm_tile);
    xab_dfree(ctx, pl->tile_ptr);
    xab_dfree(ctx, pl->tile_blk);
    xab_dfree(ctx, pl->tile_slot);
    xab_dfree(ctx, pl->tile_minblk);
    xab_dfree(ctx, pl->partial);
    xab_dfree(ctx, pl->xcb_rowptr);
    xab_dfree(ctx, pl->xcb_gbase);
    xab_dfree(ctx, pl->s3_ci);
    xab_dfree(ctx, pl->s3_dense);
    xab_dfree(ctx, pl->s3_ch0);
    xab_dfree(ctx, pl->s3_cw);
    xab_dfree(ctx, pl->s3_coff);
    xab_dfree(ctx, pl->s3_cols);
    xab_dfree(ctx, pl->s3_v64);
    xab_dfree(ctx, pl->s3_v32);
    xab_sell_free(ctx, &pl->sell);
    xab_dfree(ctx, pl->bcsr_brp);
    xab_dfree(ctx, pl->bcsr_bci);
    xab_dfree(ctx, pl->bcsr_mask);
    xab_dfree(ctx, pl->bcsr_val64);
    xab_dfree(ctx, pl->bcsr_val32);
    xab_dfree(ctx, pl->xcb_mask);
    xab_dfree(ctx, pl->xcb_colind);
    xab_dfree(ctx, pl->xcb_val64);
    xab_dfree(ctx, pl->xcb_val32);
    xab_dfree(ctx, pl->xcb_row_lo);
    xab_dfree(ctx, pl->xcb_tile_row);
    xab_dfree(ctx, pl->xcb_carry_row);
    xab_dfree(ctx, pl->xcb_tail_row);
    xab_dfree(ctx, pl->xcb_carry_val);
    xab_dfree(ctx, pl->xcb_tail_val);
    xab_dfree(ctx, pl->xcb_Y);
    xab_dfree(ctx, pl->xcb_colind32);
    xab_dfree(ctx, pl->xcb_row_lo32);
    xab_dfree(ctx, pl->xcb_tile_row32);
    xab_dfree(ctx, pl->xcb_carry_row32);
    xab_dfree(ctx, pl->xcb_tail_row32);
    xab_dfree(ctx, pl->xcb_carry_val32);
    xab_dfree(ctx, pl->xcb_tail_val32);
}

// device bytes of the plan's own arrays
static size_t plan_device_bytes(const xab_plan *pl) {
    const xab_ctx *c = pl->ctx;
    const void *arrays[] = {pl->b, pl->row_lo, pl->tile_row, pl->carry_row, pl->carry_val, pl->tail_val,
                            pl->tail_row, pl->tm_ptr, pl->tm_tile, pl->tile_ptr, pl->tile_blk, pl->tile_slot,
                            pl->tile_minblk, pl->partial, pl->xcb_rowptr, pl->xcb_gbase, pl->s3_ci, pl->s3_dense,
                            pl->s3_ch0, pl->s3_cw, pl->s3_coff, pl->s3_cols, pl->s3_v64, pl->s3_v32,
                            pl->sell.perm, pl->sell.rlen, pl->sell.clen, pl->sell.cptr, pl->sell.cols,
                            pl->sell.val64, pl->sell.val32, pl->bcsr_brp, pl->bcsr_bci, pl->bcsr_mask,
                            pl->bcsr_val64, pl->bcsr_val32, pl->xcb_mask, pl->xcb_colind, pl->xcb_val64,
                            pl->xcb_val32, pl->xcb_row_lo, pl->xcb_tile_row, pl->xcb_carry_row, pl->xcb_tail_row,
                            pl->xcb_carry_val, pl->xcb_tail_val, pl->xcb_Y, pl->xcb_colind32, pl->xcb_row_lo32,
                            pl->xcb_tile_row32, pl->xcb_carry_row32, pl->xcb_tail_row32, pl->xcb_carry_val32,
                            pl->xcb_tail_val32};
    size_t t = xab_dbytes(c, pl->xcb_ysum);
    for (const xab_plan *q : pl->xcb_sub) t += plan_device_bytes(q);
    for (const void *p : arrays) t += xab_dbytes(c, p);
    return t;
}

#define ALLOC(ptr, T, count)                                              \
    do {                                                                  \
        (ptr) = (T *)xab_dalloc(ctx, sizeof(T) * (size_t)(count));        \
        if (!(ptr)) {                                                     \
            free_plan_arrays(ctx, pl);                                    \
            delete pl;                                                    \
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");         \
        }                                                                 \
    } while (0)

#define CHECKED(call)                                \
    do {                                             \
        int _s = (call);                             \
        if (_s != XAB_OK) {                          \
            free_plan_arrays(ctx, pl);               \
            delete pl;                               \
            return _s;                               \
        }                                            \
    } while (0)

static int hip_ok(xab_ctx *ctx, hipError_t e, const char *w) { return xab_hip_check(ctx, e, w); }

void xab_sell_free(xab_ctx *ctx, xab_sell *s) {
    xab_dfree(ctx, s->perm);
    xab_dfree(ctx, s->rlen);
    xab_dfree(ctx, s->clen);
    xab_dfree(ctx, s->cptr);
    xab_dfree(ctx, s->cols);
    xab_dfree(ctx, s->val64);
    xab_dfree(ctx, s->val32);
    *s = xab_sell{};
}

int xab_sell_build(xab_ctx *ctx, const int32_t *rowptr, const int32_t *colind, const double *v64, const float *v32,
                   bool has64, bool has32, int32_t n, int64_t nnz, int32_t sigma, xab_sell *out) {
    constexpr int C = xab_plan::kSellC;
    hipStream_t st = ctx->stream;
    xab_sell &S = *out;
    S = xab_sell{};
    S.sigma = sigma;
    const int64_t nch = std::max<int64_t>(1, ((int64_t)n + C - 1) / C);
    S.nch = nch;
    S.perm = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)std::max<int32_t>(1, n));
    S.rlen = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)(nch * C));
    S.clen = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)nch);
    S.cptr = (int64_t *)xab_dalloc(ctx, sizeof(int64_t) * (size_t)(nch + 2));
    if (!S.perm || !S.rlen || !S.clen || !S.cptr) {
        xab_sell_free(ctx, &S);
        return xab_fail(ctx, XAB_E_NOMEM, "SELL layout");
    }
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(nch * C, 256)), dim3(256), 0, st, S.rlen, nch * C);
    if (n > 0) {
        int P2 = 64;
        while (P2 < sigma) P2 <<= 1;
        hipLaunchKernelGGL(k_sell_sort, dim3(grid_for(n, sigma)), dim3(P2), 0, st, rowptr, n, sigma, S.perm, S.rlen);
    }
    hipLaunchKernelGGL(k_sell_widths, dim3(grid_for(nch, 256)), dim3(256), 0, st, S.rlen, n, nch, S.clen);
    hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, st, S.clen, nch, S.cptr);
    int64_t hdr[2] = {0, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hdr, S.cptr + nch, sizeof(hdr), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        xab_sell_free(ctx, &S);
        return xab_hip_check(ctx, e, "SELL layout");
    }
    S.total = hdr[0];
    // limits: rows of at most 4096 entries (one lane sums a row) and
    // padding at most the entries themselves plus one chunk of the widest row
    if (hdr[1] > xab_plan::kSellMaxRow || hdr[0] > 2 * nnz + (int64_t)C * hdr[1]) {
        xab_sell_free(ctx, &S);
        return xab_fail(ctx, XAB_E_UNSUPPORTED, "SELL: %s",
                        hdr[1] > xab_plan::kSellMaxRow ? "a row is longer than 4096" : "padding would exceed the entries");
    }
    const size_t tot = (size_t)std::max<int64_t>(1, S.total);
    S.cols = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * tot);
    if (has64) S.val64 = (double *)xab_dalloc(ctx, sizeof(double) * tot);
    if (has32) S.val32 = (float *)xab_dalloc(ctx, sizeof(float) * tot);
    if (!S.cols || (has64 && !S.val64) || (has32 && !S.val32)) {
        xab_sell_free(ctx, &S);
        return xab_fail(ctx, XAB_E_NOMEM, "SELL copy");
    }
    hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(nch * C, 256)), dim3(256), 0, st, rowptr, colind, v64, v32, n, nch,
                       S.perm, S.rlen, S.cptr, S.clen, S.cols, S.val64, S.val32);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        xab_sell_free(ctx, &S);
        return xab_hip_check(ctx, e, "SELL fill");
    }
    return XAB_OK;
}

void xab_launch_split_bss(hipStream_t st, const int32_t *rowptr, int32_t n, int64_t T, int64_t P, int32_t *row_lo,
                          int32_t *tile_row, int32_t *carry_row) {
    hipLaunchKernelGGL(k_split_bss, dim3(grid_for(P + 1, 256)), dim3(256), 0, st, rowptr, n, T, P, row_lo, tile_row,
                       carry_row);
}

// XCB column slices: as asked, else the fewest (a power of two) that keep
// every one of a slice's 8 blocks under 262,144 columns
static int32_t xcb_slice_count(const xab_params &p, int32_t ncols) {
    if (p.xcb_slices > 0) return p.xcb_slices;
    int32_t S = 1;
    while (S < 64 && ((int64_t)ncols + 8 * (int64_t)S - 1) / (8 * (int64_t)S) > 262144) S *= 2;
    return S;
}

// A plan over the whole matrix; for XCB, of the column window [c0, c1)
// (one slice of a sliced plan).
static int build_plan(xab_ctx *ctx, const xab_matrix *A, xab_variant v, const xab_params *pp, int32_t c0, int32_t c1,
                      xab_plan **out) {
    if (!ctx || !A || !pp || !out) return XAB_E_NULL;
    *out = nullptr;
    xab_params p = *pp;
    bool symv = (v == XAB_SYM_S3 || v == XAB_SYM_ATOMIC);
    if (symv != A->sym())
        return xab_fail(ctx, XAB_E_UNSUPPORTED, symv ? "symmetric variant on a general matrix"
                                                     : "general variant on lower-stored symmetric matrix");
    auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
    switch (v) {
        case XAB_ROW:
        case XAB_SYM_ATOMIC:
            if (!pow2(p.lanes_per_row) || p.lanes_per_row > 64)
                return xab_fail(ctx, XAB_E_UNSUPPORTED, "lanes_per_row must be a power of two <= 64");
            break;
        case XAB_NNZ:
            if (p.tile_nnz < 64) return xab_fail(ctx, XAB_E_UNSUPPORTED, "tile_nnz < 64");
            break;
        case XAB_BSS:
        case XAB_XCB:
            if (v == XAB_XCB) {
                // 0: entries per lane chosen from the size once the plan
                // has counted its entries
                if (p.j_per_lane != 0 && (p.j_per_lane < 1 || p.j_per_lane > 32 || !pow2(p.j_per_lane)))
                    return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane must be 0 or a power of two in [1, 32]");
                if (p.xcb_slices != 0 && (!pow2(p.xcb_slices) || p.xcb_slices > 64))
                    return xab_fail(ctx, XAB_E_UNSUPPORTED, "xcb_slices must be 0 or a power of two in [1, 64]");
                break;
            }
            if (p.j_per_lane < 1 || p.j_per_lane > 32 || !pow2(p.j_per_lane))
                return xab_fail(ctx, XAB_E_UNSUPPORTED, "j_per_lane must be a power of two in [1, 32]");
            break;
        case XAB_SELL:
            if (p.tile_rows < xab_plan::kSellC || p.tile_rows > 1024 || p.tile_rows % xab_plan::kSellC != 0)
                return xab_fail(ctx, XAB_E_UNSUPPORTED, "SELL window (tile_rows) must be a multiple of 64 in [64, 1024]");
            break;
        case XAB_BCSR:
            break;
        case XAB_SYM_S3:
            if (!pow2(p.col_block) || p.col_block < 16 || p.col_block > xab::sym::kExtCap)
                return xab_fail(ctx, XAB_E_UNSUPPORTED, "col_block must be a power of two in [16, %d]",
                                xab::sym::kExtCap);
            if (p.tile_rows < 1 || p.tile_rows > xab::sym::kRowCap)
                return xab_fail(ctx, XAB_E_UNSUPPORTED, "tile_rows must be in [1, %d]", xab::sym::kRowCap);
            if (p.tile_nnz < 64) return xab_fail(ctx, XAB_E_UNSUPPORTED, "tile_nnz < 64");
            if (A->n >= xab::sym::kMaxCols)
                return xab_fail(ctx, XAB_E_UNSUPPORTED, "symmetric tiles need fewer than 2^30 - 1 rows");
            break;
        default:
            return xab_fail(ctx, XAB_E_UNSUPPORTED, "unknown variant %d", (int)v);
    }
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    xab_plan *pl = new xab_plan();
    pl->ctx = ctx;
    pl->A = A;
    pl->variant = v;
    pl->params = p;
    hipStream_t st = ctx->stream;
    const int32_t n = A->n;
    const int64_t nnz = A->nnz;

    if (v == XAB_ROW || v == XAB_SYM_ATOMIC) {
        int64_t rows_per_wg = 256 / p.lanes_per_row;
        pl->P = std::max<int64_t>(1, (n + rows_per_wg - 1) / rows_per_wg);
    } else if (v == XAB_NNZ) {
        pl->P = std::max<int64_t>(1, (nnz + p.tile_nnz - 1) / p.tile_nnz);
        ALLOC(pl->b, int32_t, pl->P + 1);
        hipLaunchKernelGGL(k_split_nnz, dim3(grid_for(pl->P + 1, 256)), dim3(256), 0, st, A->rowptr, n, nnz, pl->P,
                           pl->b);
        CHECKED(hip_ok(ctx, hipGetLastError(), "k_split_nnz"));
    } else if (v == XAB_BSS) {
        int64_t T = 256 * (int64_t)p.j_per_lane;
        pl->P = std::max<int64_t>(1, (nnz + T - 1) / T);
        ALLOC(pl->row_lo, int32_t, pl->P + 1);
        ALLOC(pl->tile_row, int32_t, pl->P + 1);
        ALLOC(pl->carry_row, int32_t, pl->P);
        ALLOC(pl->tail_row, int32_t, pl->P);
        ALLOC(pl->carry_val, double, pl->P);
        ALLOC(pl->tail_val, double, pl->P);
        hipLaunchKernelGGL(k_split_bss, dim3(grid_for(pl->P + 1, 256)), dim3(256), 0, st, A->rowptr, n, T, pl->P,
                           pl->row_lo, pl->tile_row, pl->carry_row);
        CHECKED(hip_ok(ctx, hipGetLastError(), "k_split_bss"));
    } else if (v == XAB_SELL) {
        pl->P = std::max<int64_t>(1, ((int64_t)n + xab_plan::kSellC - 1) / xab_plan::kSellC);
        const int s = xab_sell_build(ctx, A->rowptr, A->colind, A->val64, A->val32, A->has64, A->has32, n, nnz,
                                     p.tile_rows, &pl->sell);
        if (s != XAB_OK) {
            free_plan_arrays(ctx, pl);
            delete pl;
            return s;
        }
    } else if (v == XAB_BCSR) {
        constexpr int B = xab_plan::kBcsrB;
        const int64_t nbr = ((int64_t)n + B - 1) / B;
        pl->bcsr_nbr = nbr;
        pl->P = std::max<int64_t>(1, nbr);
        ALLOC(pl->bcsr_brp, int32_t, nbr + 1);
        int32_t *cnt = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)std::max<int64_t>(1, nbr));
        const int64_t ntile = (nbr + kScanTile - 1) / kScanTile;
        int32_t *sums = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (ntile + 2));
        int32_t *offs = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (ntile + 2));
        auto cleanup = [&]() {
            xab_dfree(ctx, cnt);
            xab_dfree(ctx, sums);
            xab_dfree(ctx, offs);
        };
        if (!cnt || !sums || !offs) {
            cleanup();
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "BCSR plan");
        }
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, (int32_t *)ctx->d_flag, (int64_t)1);
        if (nbr > 0)
            hipLaunchKernelGGL(k_bcsr_count, dim3((unsigned)nbr), dim3(kBcsrNT), 0, st, A->rowptr, A->colind, n, cnt,
                               ctx->d_flag);
        const unsigned g = (unsigned)std::max<int64_t>(1, ntile);
        hipLaunchKernelGGL(k_scan_tile_sums, dim3(g), dim3(256), 0, st, cnt, nbr, sums);
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, sums, (int64_t)g, offs);
        hipLaunchKernelGGL(k_scan_tile_apply, dim3(g), dim3(256), 0, st, cnt, nbr, offs, pl->bcsr_brp);
        int32_t hdr[2] = {0, 0};
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&hdr[0], pl->bcsr_brp + nbr, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hdr[1], ctx->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        cleanup();
        if (e != hipSuccess) {
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_hip_check(ctx, e, "BCSR layout");
        }
        const int64_t nb = hdr[0];
        pl->bcsr_nb = nb;
        if (hdr[1] || nb * B * B > 2 * nnz) {
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_UNSUPPORTED, "BCSR: %s",
                            hdr[1] ? "a block row has more than 4096 entries" : "the blocks would hold more than twice the entries");
        }
        const int64_t nbx = std::max<int64_t>(1, nb);
        ALLOC(pl->bcsr_bci, int32_t, nbx);
        ALLOC(pl->bcsr_mask, int32_t, nbx);
        if (A->has64) ALLOC(pl->bcsr_val64, double, nbx * B * B);
        if (A->has32) ALLOC(pl->bcsr_val32, float, nbx * B * B);
        e = hipMemsetAsync(pl->bcsr_mask, 0, sizeof(int32_t) * nbx, st);
        if (e == hipSuccess && pl->bcsr_val64) e = hipMemsetAsync(pl->bcsr_val64, 0, sizeof(double) * nbx * B * B, st);
        if (e == hipSuccess && pl->bcsr_val32) e = hipMemsetAsync(pl->bcsr_val32, 0, sizeof(float) * nbx * B * B, st);
        if (e == hipSuccess && nbr > 0 && nb > 0)
            hipLaunchKernelGGL(k_bcsr_fill, dim3((unsigned)nbr), dim3(kBcsrNT), 0, st, A->rowptr, A->colind, A->val64,
                               A->val32, n, pl->bcsr_brp, pl->bcsr_bci, pl->bcsr_mask, pl->bcsr_val64, pl->bcsr_val32);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_hip_check(ctx, e, "BCSR fill");
        }
    } else if (v == XAB_XCB && c0 == 0 && c1 == A->ncols && xcb_slice_count(p, A->ncols) > 1) {
        // column slices walked one after another, each an XCB plan of its
        // own over 8 blocks (one per XCD) of its columns; the products add
        // up in slice order through an accumulation-type sum
        const int32_t S = xcb_slice_count(p, A->ncols);
        xab_params q = p;
        q.xcb_slices = 1;
        pl->xcb_sub.assign((size_t)S, nullptr);
        for (int32_t i = 0; i < S; ++i) {
            const int32_t s0 = (int32_t)((int64_t)A->ncols * i / S), s1 = (int32_t)((int64_t)A->ncols * (i + 1) / S);
            CHECKED(build_plan(ctx, A, v, &q, s0, s1, &pl->xcb_sub[(size_t)i]));
            pl->P = std::max(pl->P, pl->xcb_sub[(size_t)i]->P);
        }
        pl->params.j_per_lane = pl->xcb_sub[0]->params.j_per_lane;
        pl->params.xcb_slices = S;
        ALLOC(pl->xcb_ysum, double, std::max<int64_t>(1, n));
    } else if (v == XAB_XCB) {
        constexpr int KB = xab_plan::kXcb;
        pl->params.xcb_slices = 1;
        pl->xcb_c0 = c0;
        pl->xcb_c1 = c1;
        ColBlocks cbk;
        for (int k = 0; k <= KB; ++k) cbk.cb[k] = (int32_t)(c0 + (int64_t)k * (c1 - c0) / KB);
        pl->P = 0;
        // per-row block counts -> per-block row pointers -> stable scatter
        int32_t *cnt = nullptr, *sums = nullptr, *offs = nullptr;
        int64_t *dbase = nullptr;
        const int64_t ntile = (n + kScanTile - 1) / kScanTile;
        ALLOC(pl->xcb_rowptr, int32_t, (int64_t)KB * (n + 1));
        cnt = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)KB * std::max<int32_t>(1, n));
        // scans of up to max(1, ntile) tile sums write one slot past them
        sums = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (ntile + 2));
        offs = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (ntile + 2));
        dbase = (int64_t *)xab_dalloc(ctx, sizeof(int64_t) * (KB + 1));
        auto free_tmp = [&]() {
            xab_dfree(ctx, cnt);
            xab_dfree(ctx, sums);
            xab_dfree(ctx, offs);
            xab_dfree(ctx, dbase);
        };
        if (!cnt || !sums || !offs || !dbase) {
            free_tmp();
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
        }
        if (n > 0) hipLaunchKernelGGL(k_xcb_count, dim3(grid_for(n, 256)), dim3(256), 0, st, A->rowptr, A->colind, n, cbk, cnt);
        for (int k = 0; k < KB; ++k) {
            const int32_t *in = cnt + (int64_t)k * n;
            int32_t *out = pl->xcb_rowptr + (int64_t)k * (n + 1);
            const unsigned g = (unsigned)std::max<int64_t>(1, ntile);
            hipLaunchKernelGGL(k_scan_tile_sums, dim3(g), dim3(256), 0, st, in, (int64_t)n, sums);
            hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, sums, (int64_t)g, offs);
            hipLaunchKernelGGL(k_scan_tile_apply, dim3(g), dim3(256), 0, st, in, (int64_t)n, offs, out);
        }
        int32_t tot[KB];
        hipError_t e = hipGetLastError();
        for (int k = 0; k < KB && e == hipSuccess; ++k)
            e = hipMemcpyAsync(&tot[k], pl->xcb_rowptr + (int64_t)k * (n + 1) + n, sizeof(int32_t),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_tmp();
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_hip_check(ctx, e, "column-block counts");
        }
        // the window's entries, and the copies of them
        int64_t wnnz = 0;
        for (int k = 0; k < KB; ++k) wnnz += tot[k];
        pl->xcb_colind = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)std::max<int64_t>(1, wnnz));
        if (A->has64) pl->xcb_val64 = (double *)xab_dalloc(ctx, sizeof(double) * (size_t)std::max<int64_t>(1, wnnz));
        if (A->has32) pl->xcb_val32 = (float *)xab_dalloc(ctx, sizeof(float) * (size_t)std::max<int64_t>(1, wnnz));
        if (!pl->xcb_colind || (A->has64 && !pl->xcb_val64) || (A->has32 && !pl->xcb_val32)) {
            free_tmp();
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
        }
        // entries per lane from the size (j_per_lane 0): the largest of 4,
        // 8, 16 and 32 that still cuts the window into at least 4096 tiles
        // (16 per CU); more entries per lane keep more gathers in flight
        if (pp->j_per_lane == 0) {
            int32_t J = 4;
            while (J < 32 && wnnz >= (int64_t)4096 * 256 * (2 * J)) J *= 2;
            pl->params.j_per_lane = J;
        }
        p.j_per_lane = pl->params.j_per_lane;
        const int64_t T = 256 * (int64_t)p.j_per_lane;
        // FP32 values: the size rule capped at 16 entries per lane (their
        // products then keep more workgroups per CU); only when the plan
        // chose J from the size and that gives a different J
        if (pp->j_per_lane == 0 && A->has32) {
            int32_t j32 = 4;
            while (j32 < 16 && wnnz >= (int64_t)4096 * 256 * (2 * j32)) j32 *= 2;
            pl->xcb_j32 = j32 < p.j_per_lane ? j32 : 0;
        }
        const int64_t T32 = 256 * (int64_t)pl->xcb_j32;
        pl->xcb_base[0] = 0;
        pl->xcb_toff[0] = 0;
        pl->xcb_toff32[0] = 0;
        for (int k = 0; k < KB; ++k) {
            if (T32 > 0) {
                pl->xcb_P32[k] = std::max<int64_t>(1, (tot[k] + T32 - 1) / T32);
                pl->xcb_toff32[k + 1] = pl->xcb_toff32[k] + pl->xcb_P32[k] + 1;
            }
            pl->xcb_base[k + 1] = pl->xcb_base[k] + tot[k];
            pl->xcb_P[k] = std::max<int64_t>(1, (tot[k] + T - 1) / T);
            pl->xcb_toff[k + 1] = pl->xcb_toff[k] + pl->xcb_P[k] + 1;
        }
        e = hipMemcpyAsync(dbase, pl->xcb_base, sizeof(int64_t) * (KB + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && n > 0)
            hipLaunchKernelGGL(k_xcb_scatter, dim3(grid_for(n, 256)), dim3(256), 0, st, A->rowptr, A->colind, A->val64,
                               A->val32, n, cbk, pl->xcb_rowptr, dbase, pl->xcb_colind, pl->xcb_val64, pl->xcb_val32);
        // each block's CSR over its non-empty rows (so no tile walks rows the
        // block does not touch), the head flags in its columns, and the
        // per-row block mask for the combine
        int32_t *crowptr = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)KB * (n + 1));
        pl->xcb_mask = (uint8_t *)xab_dalloc(ctx, (size_t)std::max<int32_t>(1, n));
        int32_t *flag = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)(n + 1));
        int32_t *pos = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)(n + 1));
        if (!flag || !pos || !crowptr || !pl->xcb_mask) e = hipErrorOutOfMemory;
        if (e == hipSuccess && n > 0)
            hipLaunchKernelGGL(k_xcb_mask, dim3(grid_for(n, 256)), dim3(256), 0, st, cnt, n, pl->xcb_mask);
        int32_t mk[KB] = {0};
        for (int k = 0; k < KB && e == hipSuccess; ++k) {
            const unsigned g = (unsigned)std::max<int64_t>(1, ntile);
            int32_t *crp = crowptr + (int64_t)k * (n + 1);
            if (n > 0) hipLaunchKernelGGL(k_nonzero_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, cnt + (int64_t)k * n, n, flag);
            hipLaunchKernelGGL(k_scan_tile_sums, dim3(g), dim3(256), 0, st, flag, (int64_t)n, sums);
            hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, sums, (int64_t)g, offs);
            hipLaunchKernelGGL(k_scan_tile_apply, dim3(g), dim3(256), 0, st, flag, (int64_t)n, offs, pos);
            hipLaunchKernelGGL(k_xcb_compress, dim3(grid_for(n + 1, 256)), dim3(256), 0, st, flag, pos,
                               pl->xcb_rowptr + (int64_t)k * (n + 1), n, crp);
            e = hipMemcpyAsync(&mk[k], pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);  // flag / pos are reused by the next block
            if (e == hipSuccess && mk[k] > 0)
                hipLaunchKernelGGL(k_xcb_flag_heads, dim3(grid_for(mk[k], 256)), dim3(256), 0, st, crp, mk[k],
                                   pl->xcb_colind + pl->xcb_base[k]);
        }
        if (e == hipSuccess) e = hipGetLastError();
        // the combine's group offsets: exclusive scans over 256-row groups
        pl->xcb_G = std::max<int64_t>(1, (n + 255) / 256);
        const int64_t G = pl->xcb_G;
        int32_t *gcnt = nullptr;
        if (e == hipSuccess) {
            pl->xcb_gbase = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)KB * (G + 1));
            gcnt = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)KB * G);
            if (!pl->xcb_gbase || !gcnt) e = hipErrorOutOfMemory;
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_xcb_group_counts, dim3((unsigned)G), dim3(256), 0, st, pl->xcb_mask, n, G, gcnt);
            const int64_t gt = (G + kScanTile - 1) / kScanTile;  // <= ntile + 1 slots of sums / offs
            for (int k = 0; k < KB; ++k) {
                hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)gt), dim3(256), 0, st, gcnt + (int64_t)k * G, G, sums);
                hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, sums, gt, offs);
                hipLaunchKernelGGL(k_scan_tile_apply, dim3((unsigned)gt), dim3(256), 0, st, gcnt + (int64_t)k * G, G,
                                   offs, pl->xcb_gbase + (int64_t)k * (G + 1));
            }
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        xab_dfree(ctx, gcnt);
        xab_dfree(ctx, flag);
        xab_dfree(ctx, pos);
        free_tmp();
        if (e != hipSuccess) xab_dfree(ctx, crowptr);
        CHECKED(hip_ok(ctx, e, "column-block scatter"));
        pl->xcb_ybase[0] = 0;
        for (int k = 0; k < KB; ++k) {
            pl->xcb_m[k] = mk[k];
            pl->xcb_ybase[k + 1] = pl->xcb_ybase[k] + mk[k];
        }
        const int64_t tt = pl->xcb_toff[KB];
        pl->xcb_row_lo = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)tt);
        pl->xcb_tile_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)tt);
        pl->xcb_carry_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)tt);
        pl->xcb_tail_row = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)tt);
        pl->xcb_carry_val = xab_dalloc(ctx, sizeof(double) * (size_t)tt);
        pl->xcb_tail_val = xab_dalloc(ctx, sizeof(double) * (size_t)tt);
        pl->xcb_Y = xab_dalloc(ctx, sizeof(double) * (size_t)std::max<int64_t>(1, pl->xcb_ybase[KB]));
        if (pl->xcb_j32) {
            const int64_t t32 = pl->xcb_toff32[KB];
            pl->xcb_row_lo32 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)t32);
            pl->xcb_tile_row32 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)t32);
            pl->xcb_carry_row32 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)t32);
            pl->xcb_tail_row32 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)t32);
            pl->xcb_carry_val32 = xab_dalloc(ctx, sizeof(double) * (size_t)t32);
            pl->xcb_tail_val32 = xab_dalloc(ctx, sizeof(double) * (size_t)t32);
            pl->xcb_colind32 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (size_t)std::max<int64_t>(1, wnnz));
        }
        const bool miss32 = pl->xcb_j32 && (!pl->xcb_row_lo32 || !pl->xcb_tile_row32 || !pl->xcb_carry_row32 ||
                                            !pl->xcb_tail_row32 || !pl->xcb_carry_val32 || !pl->xcb_tail_val32 ||
                                            !pl->xcb_colind32);
        if (!pl->xcb_row_lo || !pl->xcb_tile_row || !pl->xcb_carry_row || !pl->xcb_tail_row || !pl->xcb_carry_val ||
            !pl->xcb_tail_val || !pl->xcb_Y || miss32) {
            xab_dfree(ctx, crowptr);
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
        }
        for (int k = 0; k < KB; ++k) {
            const int64_t o = pl->xcb_toff[k];
            hipLaunchKernelGGL(k_split_bss, dim3(grid_for(pl->xcb_P[k] + 1, 256)), dim3(256), 0, st,
                               crowptr + (int64_t)k * (n + 1), (int32_t)pl->xcb_m[k], T, pl->xcb_P[k],
                               pl->xcb_row_lo + o, pl->xcb_tile_row + o, pl->xcb_carry_row + o);
            pl->P = std::max(pl->P, pl->xcb_P[k]);
            if (pl->xcb_j32) {
                const int64_t o32 = pl->xcb_toff32[k];
                hipLaunchKernelGGL(k_split_bss, dim3(grid_for(pl->xcb_P32[k] + 1, 256)), dim3(256), 0, st,
                                   crowptr + (int64_t)k * (n + 1), (int32_t)pl->xcb_m[k], T32, pl->xcb_P32[k],
                                   pl->xcb_row_lo32 + o32, pl->xcb_tile_row32 + o32, pl->xcb_carry_row32 + o32);
            }
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // crowptr is freed next
        xab_dfree(ctx, crowptr);
        CHECKED(hip_ok(ctx, e, "column-block tiles"));
        // full tiles in lane-interleaved 16-byte groups (columns and each
        // value copy; the FP32 walk's columns and values by its own J)
        if (pl->xcb_j32 && wnnz > 0) {
            e = hipMemcpyAsync(pl->xcb_colind32, pl->xcb_colind, sizeof(int32_t) * (size_t)wnnz,
                               hipMemcpyDeviceToDevice, st);
            CHECKED(hip_ok(ctx, e, "FP32 walk columns"));
        }
        auto interleave = [&](auto *&arr, int32_t J) -> hipError_t {
            using E = std::remove_reference_t<decltype(*arr)>;
            if (!arr || wnnz == 0 || J <= (int)(16 / sizeof(E))) return hipSuccess;
            E *out = (E *)xab_dalloc(ctx, sizeof(E) * (size_t)wnnz);
            if (!out) return hipErrorOutOfMemory;
            for (int k = 0; k < KB; ++k) {
                const int64_t b = pl->xcb_base[k], m = pl->xcb_base[k + 1] - b;
                if (m > 0)
                    hipLaunchKernelGGL((k_xcb_interleave<E>), dim3(grid_for(m, 256)), dim3(256), 0, st, arr + b, out + b,
                                       m, J);
            }
            hipError_t ee = hipGetLastError();
            if (ee == hipSuccess) ee = hipStreamSynchronize(st);
            xab_dfree(ctx, arr);
            arr = out;
            return ee;
        };
        const int32_t j32 = pl->xcb_j32 ? pl->xcb_j32 : p.j_per_lane;
        e = interleave(pl->xcb_colind, p.j_per_lane);
        if (e == hipSuccess) e = interleave(pl->xcb_val64, p.j_per_lane);
        if (e == hipSuccess) e = interleave(pl->xcb_val32, j32);
        if (e == hipSuccess && pl->xcb_j32) e = interleave(pl->xcb_colind32, j32);
        CHECKED(hip_ok(ctx, e, "interleaved tiles"));
    } else {  // XAB_SYM_S3
        const int32_t C = p.col_block;
        const int32_t bmax = xab::sym::kExtCap / C;
        int64_t P0 = std::max<int64_t>(1, (nnz + p.tile_nnz - 1) / p.tile_nnz);
        int32_t *b0 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (P0 + 1));
        int32_t *cnt0 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (P0 + 1));
        int32_t *off0 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (P0 + 1));
        auto free_tmp = [&]() {
            xab_dfree(ctx, b0);
            xab_dfree(ctx, cnt0);
            xab_dfree(ctx, off0);
        };
        if (!b0 || !cnt0 || !off0) {
            free_tmp();
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
        }
        hipLaunchKernelGGL(k_split_nnz, dim3(grid_for(P0 + 1, 256)), dim3(256), 0, st, A->rowptr, n, nnz, P0, b0);
        hipLaunchKernelGGL(k_sym_round, dim3(grid_for(P0 + 1, 256)), dim3(256), 0, st, b0, P0, n, p.tile_rows);
        hipLaunchKernelGGL(k_sym_pieces, dim3(grid_for(P0, 256)), dim3(256), 0, st, b0, P0, p.tile_rows, cnt0);
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, cnt0, P0, off0);
        int32_t P = 0;
        hipError_t e = hipMemcpyAsync(&P, off0 + P0, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_tmp();
            delete pl;
            return xab_hip_check(ctx, e, "sym tile count");
        }
        pl->P = P;
        pl->b = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (P + 1));
        if (!pl->b) {
            free_tmp();
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
        }
        hipLaunchKernelGGL(k_sym_fill, dim3(grid_for(P0 + 1, 256)), dim3(256), 0, st, b0, cnt0, off0, P0, n,
                           p.tile_rows, pl->b);
        (void)hipStreamSynchronize(st);
        free_tmp();
        CHECKED(hip_ok(ctx, hipGetLastError(), "sym tiles"));
        // touch map
        pl->nblk = ((int64_t)n + C - 1) / C;
        int32_t *cnt = nullptr;
        uint32_t *bitmap = nullptr;
        ALLOC(pl->tile_minblk, int32_t, P);
        ALLOC(pl->tile_ptr, int32_t, P + 1);
        cnt = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (P + 1));
        bitmap = (uint32_t *)xab_dalloc(ctx, sizeof(uint32_t) * (size_t)P * xab::sym::kLutWords);
        if (!cnt || !bitmap) {
            xab_dfree(ctx, cnt);
            xab_dfree(ctx, bitmap);
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
        }
        hipLaunchKernelGGL(k_fill_flag, dim3(1), dim3(64), 0, st, ctx->d_flag);
        hipLaunchKernelGGL(k_sym_touch, dim3((unsigned)P), dim3(256), 0, st, A->rowptr, A->colind, pl->b, (int64_t)P,
                           C, bmax, pl->tile_minblk, cnt, bitmap, ctx->d_flag);
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, cnt, (int64_t)P, pl->tile_ptr);
        int32_t hdr[2] = {0, 0};
        e = hipMemcpyAsync(&hdr[0], ctx->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&hdr[1], pl->tile_ptr + P, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || hdr[0] != 0) {
            xab_dfree(ctx, cnt);
            xab_dfree(ctx, bitmap);
            free_plan_arrays(ctx, pl);
            delete pl;
            if (e != hipSuccess) return xab_hip_check(ctx, e, "sym touch map");
            return xab_fail(ctx, XAB_E_UNSUPPORTED,
                            "transpose part too spread for the zero-block reduction (col_block %d: %s)", C,
                            (hdr[0] & kCountBad) ? "too many blocks per tile" : "block span too wide");
        }
        pl->ntouch = hdr[1];
        int64_t nt = std::max<int64_t>(1, pl->ntouch);
        ALLOC(pl->tile_blk, int32_t, nt);
        ALLOC(pl->tile_slot, int32_t, nt);
        ALLOC(pl->tm_tile, int32_t, nt);
        ALLOC(pl->tm_ptr, int32_t, pl->nblk + 1);
        hipLaunchKernelGGL(k_sym_blocks, dim3((unsigned)P), dim3(xab::sym::kLutWords), 0, st, bitmap, pl->tile_minblk,
                           pl->tile_ptr, pl->tile_blk);
        // order the (tile, block) pairs by block, then tile: a stable
        // counting sort of the per-tile lists
        std::vector<int32_t> h_tptr(P + 1), h_blk(nt), h_slot(nt), h_tm_tile(nt), h_tm_ptr(pl->nblk + 1, 0);
        std::vector<int32_t> h_b(P + 1);
        e = hipMemcpyAsync(h_tptr.data(), pl->tile_ptr, sizeof(int32_t) * (P + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_blk.data(), pl->tile_blk, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_b.data(), pl->b, sizeof(int32_t) * (P + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        xab_dfree(ctx, cnt);
        xab_dfree(ctx, bitmap);
        CHECKED(hip_ok(ctx, e, "touch map read-back"));
        // LDS the kernel needs: most rows, most touched blocks, widest block span
        int32_t own = 1, nbmax = 0, span = 1;
        for (int32_t t = 0; t < P; ++t) {
            own = std::max(own, h_b[t + 1] - h_b[t]);
            int32_t k = h_tptr[t + 1] - h_tptr[t];
            nbmax = std::max(nbmax, k);
            if (k > 0) span = std::max(span, h_blk[h_tptr[t + 1] - 1] - h_blk[h_tptr[t]] + 1);
        }
        pl->s3_own_cap = own;
        pl->s3_ext_cap = nbmax * C;
        pl->s3_lut_cap = (span + 7) / 8 * 8;
        const size_t lds = xab::sym::lds_bytes(pl->s3_own_cap, pl->s3_ext_cap, pl->s3_lut_cap, 8);
        if (lds > (size_t)xab::sym::kLdsCap) {
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_UNSUPPORTED, "symmetric tile needs %zu bytes of LDS (col_block %d)", lds, C);
        }
        for (int64_t q = 0; q < pl->ntouch; ++q) h_tm_ptr[h_blk[q] + 1]++;
        for (int64_t c = 0; c < pl->nblk; ++c) h_tm_ptr[c + 1] += h_tm_ptr[c];
        std::vector<int32_t> fill(h_tm_ptr.begin(), h_tm_ptr.end() - 1);
        for (int32_t t = 0; t < P; ++t)
            for (int32_t q = h_tptr[t]; q < h_tptr[t + 1]; ++q) {
                int32_t slot = fill[h_blk[q]]++;
                h_tm_tile[slot] = t;
                h_slot[q] = slot;
            }
        e = hipMemcpyAsync(pl->tm_ptr, h_tm_ptr.data(), sizeof(int32_t) * (pl->nblk + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl->tm_tile, h_tm_tile.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl->tile_slot, h_slot.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        CHECKED(hip_ok(ctx, e, "touch map upload"));
        pl->partial_elem = 8;
        pl->partial = xab_dalloc(ctx, (size_t)nt * C * 8);
        if (!pl->partial) {
            free_plan_arrays(ctx, pl);
            delete pl;
            return xab_fail(ctx, XAB_E_NOMEM, "partial buffer");
        }
        // the walk: sliced (lane = row, chunks of 64 rows padded to their
        // longest row) when the padding stays within a quarter of the entries
        // and no row is longer than the sliced walk's serial row sum allows,
        // else the stream walk over the CSR entries
        ALLOC(pl->s3_ch0, int32_t, P + 1);
        {
            int32_t *cnt1 = (int32_t *)xab_dalloc(ctx, sizeof(int32_t) * (P + 1));
            if (!cnt1) {
                free_plan_arrays(ctx, pl);
                delete pl;
                return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
            }
            hipLaunchKernelGGL(k_sym_nch, dim3(grid_for(P, 256)), dim3(256), 0, st, pl->b, (int64_t)P, cnt1);
            hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, cnt1, (int64_t)P, pl->s3_ch0);
            int32_t nch = 0;
            e = hipMemcpyAsync(&nch, pl->s3_ch0 + P, sizeof(int32_t), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            xab_dfree(ctx, cnt1);
            CHECKED(hip_ok(ctx, e, "sym chunk count"));
            pl->s3_nch = nch;
        }
        const int64_t nch = std::max<int64_t>(1, pl->s3_nch);
        ALLOC(pl->s3_cw, int32_t, nch);
        ALLOC(pl->s3_coff, int64_t, nch + 1);
        int64_t padded = 0;
        int widest = 0;
        {
            int64_t *csz = (int64_t *)xab_dalloc(ctx, sizeof(int64_t) * nch);
            if (!csz) {
                free_plan_arrays(ctx, pl);
                delete pl;
                return xab_fail(ctx, XAB_E_NOMEM, "plan allocation");
            }
            hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, (int32_t *)ctx->d_flag, (int64_t)1);
            if (P > 0)
                hipLaunchKernelGGL(k_sym_widths, dim3((unsigned)P), dim3(64), 0, st, A->rowptr, pl->b, pl->s3_ch0,
                                   pl->s3_cw, csz, ctx->d_flag);
            hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, csz, pl->s3_nch, pl->s3_coff);
            e = hipMemcpyAsync(&padded, pl->s3_coff + pl->s3_nch, sizeof(int64_t), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipMemcpyAsync(&widest, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            xab_dfree(ctx, csz);
            CHECKED(hip_ok(ctx, e, "sym chunk widths"));
        }
        pl->s3_walk = xab::sym::sliced(nnz, padded, widest) ? 1 : 0;
        pl->s3_padded = padded;
        if (pl->s3_walk) {
            const int64_t tot = std::max<int64_t>(1, padded);
            ALLOC(pl->s3_cols, int32_t, tot);
            if (A->has64) ALLOC(pl->s3_v64, double, tot);
            if (A->has32) ALLOC(pl->s3_v32, float, tot);
            if (P > 0)
                hipLaunchKernelGGL(k_sym_slice_fill, dim3((unsigned)P), dim3(64), 0, st, A->rowptr, A->colind,
                                   A->val64, A->val32, pl->b, pl->s3_ch0, pl->s3_cw, pl->s3_coff, pl->s3_cols,
                                   pl->s3_v64, pl->s3_v32);
            CHECKED(hip_ok(ctx, hipGetLastError(), "sliced copy"));
        } else {
            // flagged copy of the columns and the per-tile "no empty row" marks
            ALLOC(pl->s3_ci, int32_t, std::max<int64_t>(1, nnz));
            ALLOC(pl->s3_dense, uint8_t, std::max<int64_t>(1, P));
            if (nnz > 0) {
                e = hipMemcpyAsync(pl->s3_ci, A->colind, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, st);
                CHECKED(hip_ok(ctx, e, "column copy"));
                hipLaunchKernelGGL(k_flag_row_heads, dim3(grid_for(n, 256)), dim3(256), 0, st, A->rowptr, n,
                                   pl->s3_ci);
                if (P > 0)
                    hipLaunchKernelGGL(k_sym_defer, dim3((unsigned)P), dim3(256), 0, st, A->rowptr, A->colind, pl->b,
                                       pl->s3_ci);
            }
            if (P > 0)
                hipLaunchKernelGGL(k_tile_dense, dim3(grid_for(P, 256)), dim3(256), 0, st, A->rowptr, pl->b,
                                   (int64_t)P, pl->s3_dense);
            CHECKED(hip_ok(ctx, hipGetLastError(), "flagged columns"));
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_plan_arrays(ctx, pl);
        delete pl;
        return xab_hip_check(ctx, e, "plan build");
    }
    *out = pl;
    return XAB_OK;
}

int xab_build_plan(xab_ctx *ctx, const xab_matrix *A, xab_variant v, const xab_params *pp, xab_plan **out) {
    if (!A) return XAB_E_NULL;
    return build_plan(ctx, A, v, pp, 0, A->ncols, out);
}

extern "C" {

int xab_plan_fixed(xab_ctx *ctx, const xab_matrix *A, xab_variant v, const xab_params *p, xab_plan **plan) {
    return xab_build_plan(ctx, A, v, p, plan);
}

int64_t xab_plan_bytes(const xab_plan *pl) { return pl ? (int64_t)plan_device_bytes(pl) : -1; }

void xab_plan_destroy(xab_plan *pl) {
    if (!pl) return;
    (void)hipStreamSynchronize(pl->ctx->stream);
    free_plan_arrays(pl->ctx, pl);
    delete pl;
}

int xab_plan_refresh(xab_plan *pl) {
    if (!pl) return XAB_E_NULL;
    xab_ctx *ctx = pl->ctx;
    xab_matrix *A = const_cast<xab_matrix *>(pl->A);
    hipStream_t st = ctx->stream;
    const int32_t n = A->n;
    const int64_t nnz = A->nnz;
    XAB_HIP(ctx, hipSetDevice(ctx->device));
    XAB_HIP(ctx, hipStreamSynchronize(st));  // no product of this plan still reads the copies
    // the cached Jacobi diagonal follows the values (the next solve recomputes it)
    xab_dfree(ctx, A->diag64);
    xab_dfree(ctx, A->diag32);
    A->diag64 = nullptr;
    A->diag32 = nullptr;
    const double *v64 = A->has64 ? A->val64 : nullptr;
    const float *v32 = A->has32 ? A->val32 : nullptr;
    hipError_t e = hipSuccess;
    for (xab_plan *q : pl->xcb_sub) {
        const int s = xab_plan_refresh(q);
        if (s != XAB_OK) return s;
    }
    if (pl->variant == XAB_XCB && nnz > 0 && pl->xcb_colind) {
        // values into block order (the plan's per-block row pointers and
        // block bases), then into the stored tile layout
        constexpr int KB = xab_plan::kXcb;
        ColBlocks cbk;
        for (int k = 0; k <= KB; ++k)
            cbk.cb[k] = (int32_t)(pl->xcb_c0 + (int64_t)k * (pl->xcb_c1 - pl->xcb_c0) / KB);
        int64_t *dbase = (int64_t *)xab_dalloc(ctx, sizeof(int64_t) * (KB + 1));
        double *t64 = pl->xcb_val64 ? (double *)xab_dalloc(ctx, sizeof(double) * (size_t)nnz) : nullptr;
        float *t32 = pl->xcb_val32 ? (float *)xab_dalloc(ctx, sizeof(float) * (size_t)nnz) : nullptr;
        if (!dbase || (pl->xcb_val64 && !t64) || (pl->xcb_val32 && !t32)) e = hipErrorOutOfMemory;
        if (e == hipSuccess)
            e = hipMemcpyAsync(dbase, pl->xcb_base, sizeof(int64_t) * (KB + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_xcb_scatter, dim3(grid_for(n, 256)), dim3(256), 0, st, A->rowptr, A->colind,
                               t64 ? v64 : nullptr, t32 ? v32 : nullptr, n, cbk, pl->xcb_rowptr, dbase, nullptr, t64,
                               t32);
            for (int k = 0; k < KB; ++k) {
                const int64_t b = pl->xcb_base[k], m = pl->xcb_base[k + 1] - b;
                if (m <= 0) continue;
                if (t64)
                    hipLaunchKernelGGL((k_xcb_interleave<double>), dim3(grid_for(m, 256)), dim3(256), 0, st, t64 + b,
                                       pl->xcb_val64 + b, m, pl->params.j_per_lane);
                if (t32)
                    hipLaunchKernelGGL((k_xcb_interleave<float>), dim3(grid_for(m, 256)), dim3(256), 0, st, t32 + b,
                                       pl->xcb_val32 + b, m, pl->xcb_j32 ? pl->xcb_j32 : pl->params.j_per_lane);
            }
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        xab_dfree(ctx, dbase);
        xab_dfree(ctx, t64);
        xab_dfree(ctx, t32);
    } else if (pl->variant == XAB_SELL && pl->sell.nch > 0) {
        const xab_sell &S = pl->sell;
        hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(S.nch * xab_plan::kSellC, 256)), dim3(256), 0, st, A->rowptr,
                           A->colind, S.val64 ? v64 : nullptr, S.val32 ? v32 : nullptr, n, S.nch, S.perm, S.rlen,
                           S.cptr, S.clen, nullptr, S.val64, S.val32);
        e = hipGetLastError();
    } else if (pl->variant == XAB_BCSR && pl->bcsr_nb > 0) {
        // the blocks are sums of their entries: cleared, then refilled (the
        // block columns and position masks come out as before)
        constexpr int B = xab_plan::kBcsrB;
        const int64_t nb = pl->bcsr_nb, nbr = pl->bcsr_nbr;
        if (pl->bcsr_val64) hipLaunchKernelGGL((k_fill_zero<double>), dim3(grid_for(nb * B * B, 256)), dim3(256), 0, st,
                                               pl->bcsr_val64, nb * B * B);
        if (pl->bcsr_val32) hipLaunchKernelGGL((k_fill_zero<float>), dim3(grid_for(nb * B * B, 256)), dim3(256), 0, st,
                                               pl->bcsr_val32, nb * B * B);
        if (nbr > 0)
            hipLaunchKernelGGL(k_bcsr_fill, dim3((unsigned)nbr), dim3(kBcsrNT), 0, st, A->rowptr, A->colind,
                               pl->bcsr_val64 ? v64 : nullptr, pl->bcsr_val32 ? v32 : nullptr, n, pl->bcsr_brp,
                               pl->bcsr_bci, pl->bcsr_mask, pl->bcsr_val64, pl->bcsr_val32);
        e = hipGetLastError();
    } else if (pl->variant == XAB_SYM_S3 && pl->s3_walk && pl->P > 0) {
        hipLaunchKernelGGL(k_sym_slice_fill, dim3((unsigned)pl->P), dim3(64), 0, st, A->rowptr, A->colind,
                           pl->s3_v64 ? v64 : nullptr, pl->s3_v32 ? v32 : nullptr, pl->b, pl->s3_ch0, pl->s3_cw,
                           pl->s3_coff, nullptr, pl->s3_v64, pl->s3_v32);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipErrorOutOfMemory) return xab_fail(ctx, XAB_E_NOMEM, "plan refresh buffers");
    return e == hipSuccess ? XAB_OK : xab_hip_check(ctx, e, "plan refresh");
}

int xab_plan_info(const xab_plan *pl, xab_variant *v, xab_params *p) {
    if (!pl) return XAB_E_NULL;
    if (v) *v = pl->variant;
    if (p) *p = pl->params;
    return XAB_OK;
}

int xab_plan_array(const xab_plan *pl, int32_t which, int32_t *h_out, int64_t *len) {
    if (!pl || !len) return XAB_E_NULL;
    const int32_t *src = nullptr;
    int64_t m = 0;
    switch (which) {
        case 0: src = pl->b; m = pl->b ? pl->P + 1 : 0; break;
        case 1: src = pl->row_lo; m = pl->row_lo ? pl->P + 1 : 0; break;
        case 2: src = pl->tile_row; m = pl->tile_row ? pl->P + 1 : 0; break;
        case 3: src = pl->carry_row; m = pl->carry_row ? pl->P : 0; break;
        case 4: src = pl->tm_ptr; m = pl->tm_ptr ? pl->nblk + 1 : 0; break;
        case 5: src = pl->tm_tile; m = pl->tm_tile ? pl->ntouch : 0; break;
        case 6: src = pl->tile_ptr; m = pl->tile_ptr ? pl->P + 1 : 0; break;
        case 7: src = pl->tile_blk; m = pl->tile_blk ? pl->ntouch : 0; break;
        case 8: src = pl->tile_slot; m = pl->tile_slot ? pl->ntouch : 0; break;
        case 9: src = pl->xcb_rowptr; m = pl->xcb_rowptr ? (int64_t)xab_plan::kXcb * (pl->A->n + 1) : 0; break;
        case 10: src = pl->xcb_colind; m = pl->xcb_colind ? pl->xcb_base[xab_plan::kXcb] : 0; break;
        case 11: src = pl->sell.perm; m = pl->sell.perm ? pl->A->n : 0; break;
        case 12: src = pl->sell.rlen; m = pl->sell.rlen ? pl->A->n : 0; break;
        case 13: src = pl->sell.clen; m = pl->sell.clen ? pl->sell.nch : 0; break;
        case 14: src = pl->sell.cols; m = pl->sell.cols ? pl->sell.total : 0; break;
        case 15: src = pl->bcsr_brp; m = pl->bcsr_brp ? pl->bcsr_nbr + 1 : 0; break;
        case 16: src = pl->bcsr_bci; m = pl->bcsr_bci ? pl->bcsr_nb : 0; break;
        case 17: src = pl->bcsr_mask; m = pl->bcsr_mask ? pl->bcsr_nb : 0; break;
        case 18: src = pl->s3_ci; m = pl->s3_ci ? pl->A->nnz : 0; break;
        case 19: src = pl->s3_cols ? pl->s3_ch0 : nullptr; m = pl->s3_cols ? pl->P + 1 : 0; break;
        case 20: src = pl->s3_cols ? pl->s3_cw : nullptr; m = pl->s3_cols ? pl->s3_nch : 0; break;
        case 21: src = pl->s3_cols; m = pl->s3_cols ? pl->s3_padded : 0; break;
        default: return XAB_E_SHAPE;
    }
    *len = m;
    if (!h_out || m == 0) return XAB_OK;
    xab_ctx *ctx = pl->ctx;
    XAB_HIP(ctx, hipMemcpyAsync(h_out, src, sizeof(int32_t) * m, hipMemcpyDeviceToHost, ctx->stream));
    XAB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (which == 10 && pl->params.j_per_lane > 4) {
        // the copy keeps full tiles in lane-interleaved groups of 4: report block order
        const int64_t TT = 256 * (int64_t)pl->params.j_per_lane, J = pl->params.j_per_lane, G = 4;
        std::vector<int32_t> t((size_t)TT);
        for (int k = 0; k < xab_plan::kXcb; ++k) {
            const int64_t b = pl->xcb_base[k], nk = pl->xcb_base[k + 1] - b;
            for (int64_t tile = 0; tile < nk / TT; ++tile) {
                int32_t *blk = h_out + b + tile * TT;
                for (int64_t r = 0; r < TT; ++r) {
                    const int64_t lt = r / J, q = r % J;
                    t[(size_t)r] = blk[(q / G) * 256 * G + lt * G + q % G];
                }
                std::copy(t.begin(), t.end(), blk);
            }
        }
    }
    return XAB_OK;
}

}  // extern "C"
