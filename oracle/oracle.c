/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Serial, plain FP64, written for readability against the paper:
 *   SpMV on CRS (section 3.2.2 and 4.2), symmetric SpMV from one stored
 *   triangle (section 3.2.2, third implementation; section 4.2 storage), the
 *   integer work splits behind the nnz-based decomposition and the branchless
 *   segmented scan (section 3.2.2), restarted GMRES(m) and BiCGStab
 *   (section 2.2 solver list, section 4.3 conditions), the true-residual
 *   check of the accuracy policy (section 3.3.2), and the learned selector's
 *   MLP (not in the paper).
 * Build with -ffp-contract=off: the compensated sums rely on every rounding
 * the source writes.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ SpMV */

/* Error-free transformations (Ogita, Rump & Oishi 2005): a + b = x + y and
 * a * b = x + y exactly. */
static inline void two_sum(double a, double b, double *x, double *y) {
    *x = a + b;
    double z = *x - a;
    *y = (a - (*x - z)) + (b - z);
}
static inline void two_prod(double a, double b, double *x, double *y) {
    *x = a * b;
    *y = fma(a, b, -*x);
}

/* One CRS row: Dot2 of (val, x[col]) and the absolute sum that scales the
 * tolerance. An empty row gives exactly 0. */
static void row_dot2(const int32_t *colind, const double *val, int64_t k0, int64_t k1,
                     const double *x, double *y, double *s) {
    double p = 0.0, c = 0.0, a = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        double h, r, q;
        two_prod(val[k], x[colind[k]], &h, &r);
        two_sum(p, h, &p, &q);
        c += q + r;
        a += fabs(val[k] * x[colind[k]]);
    }
    *y = p + c;
    *s = a;
}

/* y = A x for A in CRS (rowptr, colind, val): the plain definition that
 * every SpMV implementation of section 3.2.2 computes. */
void orc_spmv_csr(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                  const double *x, double *y, double *s) {
    for (int64_t i = 0; i < n; ++i) {
        double si;
        row_dot2(colind, val, rowptr[i], rowptr[i + 1], x, &y[i], &si);
        if (s) s[i] = si;
    }
}

void orc_spmv_rows(int64_t nsample, const int64_t *rows, const int32_t *rowptr,
                   const int32_t *colind, const double *val, const double *x, double *y, double *s) {
    for (int64_t t = 0; t < nsample; ++t) {
        int64_t i = rows[t];
        double si;
        row_dot2(colind, val, rowptr[i], rowptr[i + 1], x, &y[t], &si);
        if (s) s[t] = si;
    }
}

/* ------------------------------------------------------------ symmetric */

/* A = L + L_strict^T.  L holds row i's entries with col <= i.  Row i of A
 * is (row i of L) merged with (column i of L_strict), sorted by column. */
int64_t orc_sym_expand(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                       int32_t *rowptr_f, int32_t *colind_f, double *val_f) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            cnt[i] += 1;
            if (colind[k] != i) cnt[colind[k]] += 1;
        }
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; ++i) nnz += cnt[i];
    if (!rowptr_f) { free(cnt); return nnz; }
    rowptr_f[0] = 0;
    for (int64_t i = 0; i < n; ++i) rowptr_f[i + 1] = (int32_t)(rowptr_f[i] + cnt[i]);
    /* fill: for each row i, first the transposed entries (j' > i come from
     * later rows, so walk rows in order and append), then sort per row. */
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) pos[i] = rowptr_f[i];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int64_t j = colind[k];
            colind_f[pos[i]] = (int32_t)j; val_f[pos[i]] = val[k]; pos[i]++;
            if (j != i) { colind_f[pos[j]] = (int32_t)i; val_f[pos[j]] = val[k]; pos[j]++; }
        }
    /* insertion sort each row by column (rows are short) */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t a = rowptr_f[i] + 1; a < rowptr_f[i + 1]; ++a) {
            int32_t c = colind_f[a]; double v = val_f[a];
            int64_t b = a - 1;
            while (b >= rowptr_f[i] && colind_f[b] > c) {
                colind_f[b + 1] = colind_f[b]; val_f[b + 1] = val_f[b]; --b;
            }
            colind_f[b + 1] = c; val_f[b + 1] = v;
        }
    }
    free(pos);
    free(cnt);
    return nnz;
}

/* Symmetric SpMV from lower storage: expand, then the plain CRS product. */
int orc_spmv_sym(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 const double *x, double *y, double *s) {
    int64_t nnz = orc_sym_expand(n, rowptr, colind, val, NULL, NULL, NULL);
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!rp || !ci || !v) { free(rp); free(ci); free(v); return -1; }
    orc_sym_expand(n, rowptr, colind, val, rp, ci, v);
    orc_spmv_csr(n, rp, ci, v, x, y, s);
    free(rp); free(ci); free(v);
    return 0;
}

/* ---------------------------------------------------------------- plans */

/* smallest r in [0, n] with rowptr[r] >= target */
static int64_t lower_bound_rp(int64_t n, const int32_t *rowptr, int64_t target) {
    int64_t lo = 0, hi = n + 1;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (rowptr[mid] >= target) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* largest r in [0, n] with rowptr[r] <= target */
static int64_t last_le_rp(int64_t n, const int32_t *rowptr, int64_t target) {
    int64_t lo = 0, hi = n + 1;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (rowptr[mid] <= target) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

int64_t orc_nparts(int64_t nnz, int64_t T) {
    int64_t P = (nnz + T - 1) / T;
    return P < 1 ? 1 : P;
}

/* Load-balanced row decomposition (the paper's non-zero elements based
 * method): part p gets whole rows [b_p, b_{p+1}) holding about nnz/P
 * entries.  b_p = first row whose start is at or after floor(p*nnz/P), so a
 * row straddling that target stays in the earlier part; b_0 = 0, b_P = n. */
void orc_plan_nnz(int64_t n, const int32_t *rowptr, int64_t P, int32_t *b) {
    int64_t nnz = n > 0 ? rowptr[n] : 0;
    b[0] = 0;
    for (int64_t p = 1; p < P; ++p) b[p] = (int32_t)lower_bound_rp(n, rowptr, (p * nnz) / P);
    b[P] = (int32_t)n;
}

/* Branchless segmented scan split: tile t covers entries [tT, (t+1)T).
 *   row_lo[t]    first row starting at or after tT (row_lo[P] = n): the
 *                rows whose first entry lies in tile t, empty rows included
 *   tile_row[t]  the row holding entry tT (largest r with rowptr_r <= tT)
 *   carry_row[t] tile_row[t] if that row began in an earlier tile, else -1 */
void orc_plan_bss(int64_t n, const int32_t *rowptr, int64_t T, int64_t P, int32_t *row_lo,
                  int32_t *tile_row, int32_t *carry_row) {
    for (int64_t t = 0; t < P; ++t) {
        int64_t e = t * T;
        row_lo[t] = (int32_t)lower_bound_rp(n, rowptr, e);
        int64_t tr = last_le_rp(n, rowptr, e);
        if (tr > n - 1) tr = n - 1; /* only when the matrix has no entries */
        if (tr < 0) tr = 0;
        tile_row[t] = (int32_t)tr;
        carry_row[t] = (n > 0 && rowptr[tr] < e) ? (int32_t)tr : -1;
    }
    row_lo[P] = (int32_t)n;
    tile_row[P] = (int32_t)n;
}

/* Symmetric tiles: the nnz-based split of the stored lower triangle into
 * P0 = ceil(nnz/T) parts; when Rmax >= 256 every inner part boundary moves
 * to the nearest multiple of 256 rows (at most n), parts left empty by that
 * are dropped (unless the split has a single part), and a part of R rows is
 * cut into k = ceil(u/g) pieces of whole 256-row groups (u = ceil(R/256)
 * groups, at most g = floor(Rmax/256) per piece) starting at
 * b + 256 floor(i u / k); when Rmax < 256 the boundaries stay where the
 * split put them and a part is cut into k = ceil(R/Rmax) pieces at
 * b + floor(i R / k).  Returns the tile count; b (P + 1 entries) may be
 * null. */
static int64_t sym_tiles(int64_t n, const int32_t *rowptr, int64_t T, int64_t Rmax, int32_t *b) {
    int64_t nnz = n > 0 ? rowptr[n] : 0;
    int64_t P0 = orc_nparts(nnz, T);
    int32_t *b0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P0 + 1));
    orc_plan_nnz(n, rowptr, P0, b0);
    const int64_t g = Rmax / 256;
    if (g >= 1)
        for (int64_t p = 1; p < P0; ++p) {
            int64_t r = (((int64_t)b0[p] + 128) / 256) * 256;
            b0[p] = (int32_t)(r < n ? r : n);
        }
    int64_t q = 0;
    for (int64_t p = 0; p < P0; ++p) {
        int64_t R = b0[p + 1] - b0[p];
        if (R == 0 && P0 > 1) continue;
        if (g >= 1) {
            int64_t u = (R + 255) / 256, k = (u + g - 1) / g;
            if (k < 1) k = 1;
            for (int64_t i = 0; i < k; ++i, ++q)
                if (b) b[q] = (int32_t)(b0[p] + 256 * ((i * u) / k));
        } else {
            int64_t k = (R + Rmax - 1) / Rmax;
            if (k < 1) k = 1;
            for (int64_t i = 0; i < k; ++i, ++q)
                if (b) b[q] = (int32_t)(b0[p] + (i * R) / k);
        }
    }
    if (b) b[q] = (int32_t)n;
    free(b0);
    return q;
}

int64_t orc_plan_sym_ntiles(int64_t n, const int32_t *rowptr, int64_t T, int64_t Rmax) {
    return sym_tiles(n, rowptr, T, Rmax, NULL);
}

void orc_plan_sym_tiles(int64_t n, const int32_t *rowptr, int64_t T, int64_t Rmax, int32_t *b) {
    (void)sym_tiles(n, rowptr, T, Rmax, b);
}

/* Zero-element omission for the transpose reduction.  Tile p's transposed
 * entries that land below its own rows (column j < b_p) are grouped by
 * column block floor(j/C); TB_p is the set of such blocks.  Only these
 * (tile, block) pairs hold non-zero partial sums; every other region of the
 * reduction vector is zero and skipped.
 *   tm_ptr[nblk+1], tm_tile[]  pairs ordered by block, then tile ascending;
 *                              a pair's position in this order is its slot
 *   tile_ptr[P+1], tile_blk[], tile_slot[]  the same pairs per tile, blocks
 *                              ascending, with their slot
 * Returns the number of pairs; outputs may be null (count only). */
int64_t orc_plan_sym_touch(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t P,
                           const int32_t *b, int64_t C, int32_t *tm_ptr, int32_t *tm_tile,
                           int32_t *tile_ptr, int32_t *tile_blk, int32_t *tile_slot) {
    int64_t nblk = (n + C - 1) / C;
    unsigned char *mark = (unsigned char *)calloc((size_t)(nblk > 0 ? nblk : 1), 1);
    int64_t *bcount = (int64_t *)calloc((size_t)nblk + 1, sizeof(int64_t));
    int64_t total = 0;
    /* pass 1: per tile, distinct blocks -> counts */
    for (int64_t p = 0; p < P; ++p) {
        int64_t c0 = total;
        for (int64_t i = b[p]; i < b[p + 1]; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colind[k] < b[p]) {
                    int64_t c = colind[k] / C;
                    if (!mark[c]) { mark[c] = 1; total++; bcount[c]++; }
                }
        if (tile_ptr) tile_ptr[p] = (int32_t)c0;
        /* unmark */
        for (int64_t i = b[p]; i < b[p + 1]; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colind[k] < b[p]) mark[colind[k] / C] = 0;
    }
    if (!tm_ptr) { free(mark); free(bcount); return total; }
    tile_ptr[P] = (int32_t)total;
    tm_ptr[0] = 0;
    for (int64_t c = 0; c < nblk; ++c) tm_ptr[c + 1] = (int32_t)(tm_ptr[c] + bcount[c]);
    int64_t *fillpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nblk > 0 ? nblk : 1));
    for (int64_t c = 0; c < nblk; ++c) fillpos[c] = tm_ptr[c];
    /* pass 2: tiles in ascending order, so each block's tile list is ascending */
    for (int64_t p = 0; p < P; ++p) {
        int64_t q = tile_ptr[p];
        for (int64_t i = b[p]; i < b[p + 1]; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colind[k] < b[p]) {
                    int64_t c = colind[k] / C;
                    if (!mark[c]) { mark[c] = 1; tile_blk[q++] = (int32_t)c; }
                }
        /* sort this tile's blocks ascending (insertion sort, lists are short) */
        for (int64_t a = tile_ptr[p] + 1; a < q; ++a) {
            int32_t v = tile_blk[a];
            int64_t z = a - 1;
            while (z >= tile_ptr[p] && tile_blk[z] > v) { tile_blk[z + 1] = tile_blk[z]; --z; }
            tile_blk[z + 1] = v;
        }
        for (int64_t a = tile_ptr[p]; a < q; ++a) {
            int64_t c = tile_blk[a];
            mark[c] = 0;
            tm_tile[fillpos[c]] = (int32_t)p;
            tile_slot[a] = (int32_t)fillpos[c];
            fillpos[c]++;
        }
    }
    free(fillpos);
    free(mark);
    free(bcount);
    return total;
}

/* Column blocking (a data transformation of the kind the paper lists as
 * future work for SpMV, section 5): every entry goes to the block of its
 * column, keeping row order and the order inside a row. */
void orc_plan_xcb(int64_t n, int64_t ncols, const int32_t *rowptr, const int32_t *colind, int nb, int32_t *rp,
                  int32_t *ci) {
    int64_t *blk_lo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    for (int k = 0; k <= nb; ++k) blk_lo[k] = ((int64_t)k * ncols) / nb;
    int64_t pos = 0;
    for (int k = 0; k < nb; ++k) {
        int32_t *r = rp + (int64_t)k * (n + 1);
        r[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            int32_t c = 0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                if (colind[e] >= blk_lo[k] && colind[e] < blk_lo[k + 1]) {
                    ci[pos++] = colind[e];
                    c++;
                }
            r[i + 1] = r[i] + c;
        }
    }
    free(blk_lo);
}

/* The column-blocked copy's row-start flags: within each block, the first
 * entry of every row that has entries in the block gets bit 31 of its
 * column index set (the head flag of a segmented-scan format, stored in the
 * otherwise unused sign bit).  rp and ci as orc_plan_xcb wrote them. */
void orc_xcb_flag_heads(int64_t n, int nb, const int32_t *rp, int32_t *ci) {
    int64_t base = 0;
    for (int k = 0; k < nb; ++k) {
        const int32_t *r = rp + (int64_t)k * (n + 1);
        for (int64_t i = 0; i < n; ++i)
            if (r[i + 1] > r[i]) ci[base + r[i]] = (int32_t)((uint32_t)ci[base + r[i]] | 0x80000000u);
        base += r[n];
    }
}

/* The symmetric walk's column copy.  The walk issues the transposed adds
 * of a chunk of lanes * J consecutive entries (chunks start at multiples of
 * lanes * J) one slot at a time: slot k holds entry k of every lane, i.e.
 * the entries q with q % J = k.  Within one tile (rows [b_p, b_{p+1})),
 * entry q gets bit 30 when an earlier entry of its chunk and its slot has
 * the same column (then it is added after the chunk's slots, so no two
 * lanes of one add meet on a row).  The first entry of every non-empty row
 * gets bit 31.  out[nnz] receives colind with these bits. */
void orc_plan_sym_colflags(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t P, const int32_t *b,
                           int64_t lanes, int64_t J, int32_t *out) {
    const int64_t CH = lanes * J;
    for (int64_t q = 0; q < rowptr[n]; ++q) out[q] = colind[q];
    for (int64_t p = 0; p < P; ++p) {
        const int64_t s = rowptr[b[p]], e = rowptr[b[p + 1]];
        for (int64_t q = s; q < e; ++q) {
            /* the earlier entries of q's chunk and slot inside the tile */
            const int64_t lo = q - q % CH > s ? q - q % CH : s;
            int later = 0;
            for (int64_t u = q - J; u >= lo; u -= J)
                if (colind[u] == colind[q]) later = 1;
            if (later) out[q] = (int32_t)((uint32_t)out[q] | 0x40000000u);
        }
    }
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] > rowptr[i]) out[rowptr[i]] = (int32_t)((uint32_t)out[rowptr[i]] | 0x80000000u);
}

/* The symmetric product's sliced layout.  Tile p's rows [b_p, b_{p+1}) are
 * cut into chunks of `lanes` rows (the last one shorter); chunk g holds
 * rows rc .. rc + nr - 1 and has width w_g = its longest row.  Entry k of
 * the chunk's row rc + l is stored at coff_g + k * nr + l (column-major
 * with stride nr); slots past a row's end hold column -1 (value 0 in the
 * value copy).  A stored entry gets bit 30 when a lower l' of the same
 * chunk has the same column in the same slot k.  ch0[P + 1]: first chunk
 * of each tile; cw[nch], coff[nch + 1]; cols[coff_nch].  Outputs may be
 * null (sizes only).  Returns the padded size; *nch and *widest receive
 * the chunk count and the longest row. */
int64_t orc_plan_sym_slices(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t P, const int32_t *b,
                            int64_t lanes, int32_t *ch0, int32_t *cw, int64_t *coff, int32_t *cols, int64_t *nch,
                            int64_t *widest) {
    (void)n;
    int64_t g = 0, off = 0, most = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (ch0) ch0[p] = (int32_t)g;
        for (int64_t rc = b[p]; rc < b[p + 1]; rc += lanes) {
            const int64_t nr = rc + lanes < b[p + 1] ? lanes : b[p + 1] - rc;
            int64_t w = 0;
            for (int64_t l = 0; l < nr; ++l) {
                const int64_t len = rowptr[rc + l + 1] - rowptr[rc + l];
                if (len > w) w = len;
            }
            if (w > most) most = w;
            if (cw) cw[g] = (int32_t)w;
            if (coff) coff[g] = off;
            if (cols)
                for (int64_t k = 0; k < w; ++k)
                    for (int64_t l = 0; l < nr; ++l) {
                        const int64_t i = rc + l, len = rowptr[i + 1] - rowptr[i];
                        int32_t c = k < len ? colind[rowptr[i] + k] : -1;
                        if (c >= 0)
                            for (int64_t u = 0; u < l; ++u) {
                                const int64_t iu = rc + u;
                                if (k < rowptr[iu + 1] - rowptr[iu] && colind[rowptr[iu] + k] == colind[rowptr[i] + k])
                                    c = (int32_t)((uint32_t)c | 0x40000000u);
                            }
                        cols[off + k * nr + l] = c;
                    }
            off += w * nr;
            g++;
        }
    }
    if (ch0) ch0[P] = (int32_t)g;
    if (coff) coff[g] = off;
    if (nch) *nch = g;
    if (widest) *widest = most;
    return off;
}

/* Which walk the symmetric product takes: the sliced one when its padding
 * stays within a quarter of the entries and no row is longer than 4096,
 * else the walk over the CSR entry stream. */
int orc_sym_walk_sliced(int64_t nnz, int64_t padded, int64_t widest) {
    return padded <= nnz + nnz / 4 && widest <= 4096;
}

/* Block CSR (orc_plan_bcsr in oracle.h): per block row, the block columns
 * of its entries are collected, sorted and made unique; each entry then
 * finds its block by binary search and adds its value to its position. */
static int cmp_i32(const void *a, const void *b) {
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : x > y;
}

int64_t orc_plan_bcsr(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, int b,
                      int64_t *brp, int32_t *bci, uint32_t *bmask, double *bval) {
    const int64_t nbr = (n + b - 1) / b;
    int64_t total = 0;
    int64_t cap = 16;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * cap);
    if (brp) brp[0] = 0;
    for (int64_t R = 0; R < nbr; ++R) {
        const int64_t r0 = R * b, r1 = r0 + b < n ? r0 + b : n;
        const int64_t k0 = rowptr[r0], k1 = rowptr[r1];
        if (k1 - k0 > cap) {
            cap = k1 - k0;
            tmp = (int32_t *)realloc(tmp, sizeof(int32_t) * cap);
        }
        for (int64_t k = k0; k < k1; ++k) tmp[k - k0] = colind[k] / b;
        qsort(tmp, (size_t)(k1 - k0), sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t k = 0; k < k1 - k0; ++k)
            if (k == 0 || tmp[k] != tmp[k - 1]) tmp[u++] = tmp[k];
        if (bci) {
            for (int64_t q = 0; q < u; ++q) {
                bci[total + q] = tmp[q];
                bmask[total + q] = 0;
                for (int e = 0; e < b * b; ++e) bval[(total + q) * b * b + e] = 0.0;
            }
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
                    const int32_t cb = colind[k] / b;
                    int64_t lo = 0, hi = u;  /* first position with tmp[pos] >= cb */
                    while (lo < hi) {
                        const int64_t mid = (lo + hi) / 2;
                        if (tmp[mid] < cb) lo = mid + 1;
                        else hi = mid;
                    }
                    const int e = (int)(r - r0) * b + colind[k] % b;
                    bmask[total + lo] |= 1u << e;
                    bval[(total + lo) * b * b + e] += val[k];
                }
        }
        total += u;
        if (brp) brp[R + 1] = total;
    }
    free(tmp);
    return total;
}

/* Sliced ELLPACK with sorting window (SELL-C-sigma, a format the paper
 * lists among future SpMV candidates, section 5): inside every window of
 * sigma rows the rows are ordered by length, longest first (ties keep the
 * lower row first); the ordered rows are cut into chunks of C; a chunk is
 * stored column-major and padded to its longest row: entry k of the chunk's
 * lane l sits at cptr[chunk] + k*C + l.  perm[r] = original row of ordered
 * row r, rlen[r] its length, clen[chunk] the chunk width.  Returns the
 * padded size cptr[nchunks]; when cols is non-NULL also fills cols / vals
 * (padding: column 0, value 0). */
int64_t orc_plan_sell(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, int C,
                      int sigma, int32_t *perm, int64_t *cptr, int32_t *clen, int32_t *rlen, int32_t *cols,
                      double *vals) {
    for (int64_t w0 = 0; w0 < n; w0 += sigma) {
        int64_t w1 = w0 + sigma < n ? w0 + sigma : n;
        for (int64_t r = w0; r < w1; ++r) perm[r] = (int32_t)r;
        /* insertion sort: stable, longest first */
        for (int64_t r = w0 + 1; r < w1; ++r) {
            int32_t row = perm[r];
            int32_t len = rowptr[row + 1] - rowptr[row];
            int64_t q = r - 1;
            while (q >= w0 && rowptr[perm[q] + 1] - rowptr[perm[q]] < len) {
                perm[q + 1] = perm[q];
                --q;
            }
            perm[q + 1] = row;
        }
    }
    int64_t nch = (n + C - 1) / C;
    cptr[0] = 0;
    for (int64_t c = 0; c < nch; ++c) {
        int32_t wmax = 0;
        for (int64_t r = c * C; r < (c + 1) * C && r < n; ++r) {
            rlen[r] = rowptr[perm[r] + 1] - rowptr[perm[r]];
            if (rlen[r] > wmax) wmax = rlen[r];
        }
        clen[c] = wmax;
        cptr[c + 1] = cptr[c] + (int64_t)wmax * C;
    }
    if (cols) {
        for (int64_t q = 0; q < cptr[nch]; ++q) {
            cols[q] = 0;
            if (vals) vals[q] = 0.0;
        }
        for (int64_t r = 0; r < n; ++r) {
            int64_t c = r / C, l = r % C;
            for (int32_t k = 0; k < rlen[r]; ++k) {
                int64_t dst = cptr[c] + (int64_t)k * C + l, src = rowptr[perm[r]] + k;
                cols[dst] = colind[src];
                if (vals) vals[dst] = val[src];
            }
        }
    }
    return cptr[nch];
}

/* ------------------------------------------------------------- features */

/* stats: [0] n, [1] nnz, [2] sum len^2, [3] max len, [4] max |i-j|,
 *        [5] empty rows, [6] rows with len > 64, [7] sum |i-j|,
 *        [8] nnz in rows with len > 4*mean (len*n > 4*nnz)
 * feat:  log2 n, log2 nnz, mean, log2(1+var), log2 maxlen, log2(maxlen/mean),
 *        bandwidth/n, sym flag, empty fraction, long-row fraction,
 *        mean |i-j| / n, heavy-row nnz fraction.
 * log2 of a count is taken of max(count, 1). */
void orc_features(int64_t n, const int32_t *rowptr, const int32_t *colind, int sym_lower,
                  int64_t *stats, double *feat) {
    int64_t nnz = n > 0 ? rowptr[n] : 0;
    int64_t s2 = 0, mx = 0, bw = 0, empty = 0, long64 = 0, sd = 0, heavy = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t l = rowptr[i + 1] - rowptr[i];
        s2 += l * l;
        if (l > mx) mx = l;
        if (l == 0) empty++;
        if (l > 64) long64++;
        if (l * n > 4 * nnz) heavy += l;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int64_t d = i - colind[k];
            if (d < 0) d = -d;
            if (d > bw) bw = d;
            sd += d;
        }
    }
    int64_t st[9] = {n, nnz, s2, mx, bw, empty, long64, sd, heavy};
    if (stats) memcpy(stats, st, sizeof(st));
    double dn = (double)n, dnnz = (double)nnz;
    double mean = dnnz / dn;
    double var = (double)s2 / dn - mean * mean;
    if (var < 0.0) var = 0.0;
    double dmx = (double)(mx > 0 ? mx : 1);
    feat[0] = log2(dn > 1.0 ? dn : 1.0);
    feat[1] = log2(dnnz > 1.0 ? dnnz : 1.0);
    feat[2] = mean;
    feat[3] = log2(1.0 + var);
    feat[4] = log2(dmx);
    feat[5] = log2(mean > 0.0 ? dmx / mean : 1.0);
    feat[6] = (double)bw / dn;
    feat[7] = sym_lower ? 1.0 : 0.0;
    feat[8] = (double)empty / dn;
    feat[9] = (double)long64 / dn;
    feat[10] = nnz > 0 ? (double)sd / dnnz / dn : 0.0;
    feat[11] = nnz > 0 ? (double)heavy / dnnz : 0.0;
}

/* ------------------------------------------------------------------ MLP */

int64_t orc_mlp_nparams(int F, int H, int K) {
    return (int64_t)H * F + H + (int64_t)H * H + H + (int64_t)K * H + K;
}

/* o = W3 relu(W2 relu(W1 f + b1) + b2) + b3 for every row f of feat[B*F] */
void orc_mlp_forward(int F, int H, int K, const double *p, int64_t B, const double *feat, double *out) {
    const double *W1 = p, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + K * H;
    double *h1 = (double *)malloc(sizeof(double) * H), *h2 = (double *)malloc(sizeof(double) * H);
    for (int64_t s = 0; s < B; ++s) {
        const double *f = feat + s * F;
        for (int i = 0; i < H; ++i) {
            double z = b1[i];
            for (int j = 0; j < F; ++j) z += W1[i * F + j] * f[j];
            h1[i] = z > 0.0 ? z : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            double z = b2[i];
            for (int j = 0; j < H; ++j) z += W2[i * H + j] * h1[j];
            h2[i] = z > 0.0 ? z : 0.0;
        }
        for (int k = 0; k < K; ++k) {
            double z = b3[k];
            for (int j = 0; j < H; ++j) z += W3[k * H + j] * h2[j];
            out[s * K + k] = z;
        }
    }
    free(h1); free(h2);
}

/* Masked mean squared error L = (1/sum mask) sum mask (o - y)^2 and its
 * gradient by the chain rule (ReLU'(0) taken as 0). Returns L. */
double orc_mlp_loss_grad(int F, int H, int K, const double *p, int64_t B, const double *feat,
                         const double *y, const uint8_t *mask, double *grad) {
    const double *W1 = p, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + K * H;
    int64_t np = orc_mlp_nparams(F, H, K);
    memset(grad, 0, sizeof(double) * (size_t)np);
    double *gW1 = grad, *gb1 = gW1 + H * F, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H, *gb3 = gW3 + K * H;
    double cnt = 0.0;
    for (int64_t i = 0; i < B * K; ++i) cnt += mask[i] ? 1.0 : 0.0;
    if (cnt == 0.0) return 0.0;
    double *z1 = malloc(sizeof(double) * H), *h1 = malloc(sizeof(double) * H);
    double *z2 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    double *d2 = malloc(sizeof(double) * H), *d1 = malloc(sizeof(double) * H), *go = malloc(sizeof(double) * K);
    double loss = 0.0;
    for (int64_t s = 0; s < B; ++s) {
        const double *f = feat + s * F;
        for (int i = 0; i < H; ++i) {
            double z = b1[i];
            for (int j = 0; j < F; ++j) z += W1[i * F + j] * f[j];
            z1[i] = z; h1[i] = z > 0.0 ? z : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            double z = b2[i];
            for (int j = 0; j < H; ++j) z += W2[i * H + j] * h1[j];
            z2[i] = z; h2[i] = z > 0.0 ? z : 0.0;
        }
        for (int k = 0; k < K; ++k) {
            double o = b3[k];
            for (int j = 0; j < H; ++j) o += W3[k * H + j] * h2[j];
            double e = mask[s * K + k] ? o - y[s * K + k] : 0.0;
            loss += e * e;
            go[k] = 2.0 * e / cnt;
        }
        /* layer 3 */
        for (int k = 0; k < K; ++k) {
            gb3[k] += go[k];
            for (int j = 0; j < H; ++j) gW3[k * H + j] += go[k] * h2[j];
        }
        for (int j = 0; j < H; ++j) {
            double a = 0.0;
            for (int k = 0; k < K; ++k) a += W3[k * H + j] * go[k];
            d2[j] = z2[j] > 0.0 ? a : 0.0;
        }
        /* layer 2 */
        for (int i = 0; i < H; ++i) {
            gb2[i] += d2[i];
            for (int j = 0; j < H; ++j) gW2[i * H + j] += d2[i] * h1[j];
        }
        for (int j = 0; j < H; ++j) {
            double a = 0.0;
            for (int i = 0; i < H; ++i) a += W2[i * H + j] * d2[i];
            d1[j] = z1[j] > 0.0 ? a : 0.0;
        }
        /* layer 1 */
        for (int i = 0; i < H; ++i) {
            gb1[i] += d1[i];
            for (int j = 0; j < F; ++j) gW1[i * F + j] += d1[i] * f[j];
        }
    }
    free(z1); free(h1); free(z2); free(h2); free(d2); free(d1); free(go);
    return loss / cnt;
}

/* Adam (Kingma & Ba 2015), bias-corrected, step t >= 1 */
void orc_adam_step(int64_t np, double *p, const double *g, double *m, double *v, int64_t t, double lr,
                   double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Mini-batch Adam over `epochs` passes; order[e*M + i] is the sample taken
 * at position i of epoch e; a trailing short batch is kept. */
void orc_mlp_train(int F, int H, int K, double *p, int64_t M, const double *feat, const double *y,
                   const uint8_t *mask, const int32_t *order, int epochs, int batch, double lr,
                   double *loss_per_epoch) {
    int64_t np = orc_mlp_nparams(F, H, K);
    double *g = calloc((size_t)np, sizeof(double)), *m = calloc((size_t)np, sizeof(double));
    double *v = calloc((size_t)np, sizeof(double));
    double *bf = malloc(sizeof(double) * (size_t)batch * F), *by = malloc(sizeof(double) * (size_t)batch * K);
    uint8_t *bm = malloc((size_t)batch * K);
    int64_t t = 0;
    for (int e = 0; e < epochs; ++e) {
        double lsum = 0.0;
        int64_t nb = 0;
        for (int64_t s0 = 0; s0 < M; s0 += batch) {
            int64_t B = (M - s0 < batch) ? M - s0 : batch;
            for (int64_t s = 0; s < B; ++s) {
                int64_t idx = order[(int64_t)e * M + s0 + s];
                memcpy(bf + s * F, feat + idx * F, sizeof(double) * F);
                memcpy(by + s * K, y + idx * K, sizeof(double) * K);
                memcpy(bm + s * K, mask + idx * K, (size_t)K);
            }
            lsum += orc_mlp_loss_grad(F, H, K, p, B, bf, by, bm, g);
            ++nb;
            orc_adam_step(np, p, g, m, v, ++t, lr, 0.9, 0.999, 1e-8);
        }
        if (loss_per_epoch) loss_per_epoch[e] = lsum / (double)nb;
    }
    free(g); free(m); free(v); free(bf); free(by); free(bm);
}

/* -------------------------------------------------------------- Krylov */

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void spmv_plain(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                       const double *x, double *y) {
    orc_spmv_csr(n, rp, ci, v, x, y, NULL);
}

static void diag_of(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *d) {
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) d[i] += v[k];
    }
}

/* Restarted GMRES(m) (Saad & Schultz), modified Gram-Schmidt (the paper's
 * default orthogonaliser), Givens rotations r = hypot(a, b), c = a/r,
 * s = b/r.  Right preconditioning by M = diag(A) when precond == 1:
 * solve (A M^-1) u = b, x = M^-1 u.  A cycle ends early on a lucky
 * breakdown (h_{j+1,j} = 0) or when the recurrence residual meets tol.
 * Convergence is declared only on the TRUE residual ||b - A x|| / ||b||
 * computed at every restart (the accuracy policy's outer check).
 * arnoldi_err (optional) receives max over cycles of
 * ||A M^-1 V_j - V_{j+1} Hbar_j||_F / ||H||_F before the rotations. */
/* The MM ratio of eq. (1): with residual samples r(1), r(2), ... (r[0]
 * holds r(1)), R(s, t) = max over z = s-t+1 .. s of r(z) divided by the
 * min over the same window. */
double orc_mm_ratio(const double *r, int64_t s, int64_t t) {
    double mx = r[s - t], mn = r[s - t];
    for (int64_t z = s - t + 1; z <= s; ++z) {
        if (r[z - 1] > mx) mx = r[z - 1];
        if (r[z - 1] < mn) mn = r[z - 1];
    }
    return mx / mn;
}

/* Restarted GMRES(m).  With step > 0 the restart length is tuned at run
 * time in the manner of section 3.2.1 and the section 4.3 setting: after
 * every cycle the MM ratio of that cycle's residual samples (the relative
 * residual at its start and the recurrence residual after each of its
 * steps) is formed over the whole cycle, and when it is below `ratio` (the
 * residual stagnated) the next cycle's m grows by `step`, up to m_max.
 * m_hist (may be NULL) receives the m of every cycle. */
/* Orthogonalise w against the columns V_0 .. V_j (length n) by one of the
 * section 3.2.2 methods; h[0..j] receives the projection coefficients and
 * the norm of w afterwards is returned.
 *   ORC_MGS   one column at a time, each dot with the current w
 *   ORC_CGS   all dots with the incoming w, then one combined update
 *   ORC_DGKS  CGS, then CGS again when the norm fell below 1/sqrt(2) of
 *             the incoming norm (coefficients of both passes summed)
 *   ORC_BCGS  blocks of 4 columns: CGS inside a block, blocks in order */
enum { ORC_DGKS = 0, ORC_CGS = 1, ORC_MGS = 2, ORC_BCGS = 3, ORC_POLICY = 4 };

static void cgs_block(int64_t n, const double *V, int i0, int i1, double *w, double *h) {
    for (int i = i0; i < i1; ++i) h[i] = dot(n, w, V + (int64_t)i * n);
    for (int i = i0; i < i1; ++i)
        for (int64_t q = 0; q < n; ++q) w[q] -= h[i] * V[(int64_t)i * n + q];
}

static double orth_step(int ortho, int64_t n, const double *V, int j, double *w, double *h, double *h2) {
    if (ortho == ORC_MGS) {
        for (int i = 0; i <= j; ++i) cgs_block(n, V, i, i + 1, w, h);
    } else if (ortho == ORC_CGS) {
        cgs_block(n, V, 0, j + 1, w, h);
    } else if (ortho == ORC_BCGS) {
        for (int i0 = 0; i0 <= j; i0 += 4) cgs_block(n, V, i0, i0 + 4 < j + 1 ? i0 + 4 : j + 1, w, h);
    } else { /* DGKS */
        double nw = sqrt(dot(n, w, w));
        cgs_block(n, V, 0, j + 1, w, h);
        if (sqrt(dot(n, w, w)) < nw / sqrt(2.0)) {
            cgs_block(n, V, 0, j + 1, w, h2);
            for (int i = 0; i <= j; ++i) h[i] += h2[i];
        }
    }
    return sqrt(dot(n, w, w));
}

int orc_gmres_at(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 const double *b, double *x, int m0, int m_max, int step, double ratio, double tol,
                 int64_t maxiter, int precond, int64_t *info, double *dinfo, double *resid_hist,
                 double *arnoldi_err, int32_t *m_hist, int ortho_in, int32_t *policy_out) {
    /* accuracy policy (section 3.3.2): MGS when the requirement is 1e-10 or
     * tighter, else BCGS; after a fault convergence (the recurrence met the
     * threshold, the true residual did not) DGKS and a threshold narrowed
     * tenfold for the recurrence test */
    int ortho = ortho_in == ORC_POLICY ? (tol <= 1e-10 ? ORC_MGS : ORC_BCGS) : ortho_in;
    double tol_rec = tol;
    int faults = 0, stopped_by_rec = 0;
    const int m = (step > 0 && m_max > m0) ? m_max : m0; /* capacity: rows of H, columns of V */
    int cm = m0;                                          /* restart length of the current cycle */
    double *samp = malloc(sizeof(double) * (m + 1));
    double *V = malloc(sizeof(double) * (size_t)n * (m + 1));
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));   /* H[i*m + j] */
    double *H0 = calloc((size_t)(m + 1) * m, sizeof(double));  /* unrotated copy */
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *g = malloc(sizeof(double) * (m + 1)), *yv = malloc(sizeof(double) * m);
    double *w = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *dg = malloc(sizeof(double) * n);
    double *hc = malloc(sizeof(double) * (m + 1)), *hc2 = malloc(sizeof(double) * (m + 1));
    if (precond) diag_of(n, rowptr, colind, val, dg);
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    int64_t it = 0, restarts = 0;
    int status = 1;
    double aerr = 0.0, relres = 0.0;
    if (resid_hist) resid_hist[0] = NAN;
    for (;;) {
        spmv_plain(n, rowptr, colind, val, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double beta = sqrt(dot(n, r, r));
        relres = beta / bn;
        if (resid_hist && it == 0) resid_hist[0] = relres;
        if (relres <= tol) { status = 0; break; }
        if (stopped_by_rec && ortho_in == ORC_POLICY) {
            /* fault convergence */
            faults++;
            ortho = ORC_DGKS;
            tol_rec *= 0.1;
        }
        stopped_by_rec = 0;
        if (it >= maxiter) { status = 1; break; }
        if (m_hist) m_hist[restarts] = cm;
        restarts++; /* cycles started */
        for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        samp[0] = relres;
        int j, k = 0;
        for (j = 0; j < cm && it < maxiter; ++j) {
            double *vj = V + (int64_t)j * n;
            if (precond) for (int64_t i = 0; i < n; ++i) z[i] = vj[i] / dg[i];
            else memcpy(z, vj, sizeof(double) * n);
            spmv_plain(n, rowptr, colind, val, z, w);
            double hn = orth_step(ortho, n, V, j, w, hc, hc2);
            for (int i = 0; i <= j; ++i) H[i * m + j] = hc[i];
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i <= j + 1; ++i) H0[i * m + j] = H[i * m + j];
            if (hn != 0.0)
                for (int64_t q = 0; q < n; ++q) V[(int64_t)(j + 1) * n + q] = w[q] / hn;
            /* apply the earlier rotations to column j, then a new one */
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double rr = hypot(a, c);
            cs[j] = rr == 0.0 ? 1.0 : a / rr;
            sn[j] = rr == 0.0 ? 0.0 : c / rr;
            H[j * m + j] = rr;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            if (resid_hist) resid_hist[it] = fabs(g[j + 1]) / bn;
            samp[j + 1] = fabs(g[j + 1]) / bn;
            if (hn == 0.0) break;
            if (fabs(g[j + 1]) / bn <= tol_rec) { stopped_by_rec = 1; break; }
        }
        /* restart-length judgment on this cycle's samples */
        if (step > 0 && cm < m_max && k > 0 && orc_mm_ratio(samp, k + 1, k + 1) < ratio)
            cm = cm + step < m_max ? cm + step : m_max;
        if (arnoldi_err && k > 0) {
            /* || A M^-1 V_k - V_{k+1} Hbar_k ||_F / ||Hbar_k||_F (unrotated H) */
            double num = 0.0, den = 0.0;
            for (int jj = 0; jj < k; ++jj) {
                double *vj = V + (int64_t)jj * n;
                if (precond) for (int64_t i = 0; i < n; ++i) z[i] = vj[i] / dg[i];
                else memcpy(z, vj, sizeof(double) * n);
                spmv_plain(n, rowptr, colind, val, z, w);
                int top = (jj + 1 < k || H0[(jj + 1) * m + jj] != 0.0) ? jj + 1 : jj;
                for (int i = 0; i <= top && i <= m; ++i)
                    for (int64_t q = 0; q < n; ++q) w[q] -= H0[i * m + jj] * V[(int64_t)i * n + q];
                num += dot(n, w, w);
                for (int i = 0; i <= jj + 1; ++i) den += H0[i * m + jj] * H0[i * m + jj];
            }
            double e = sqrt(num) / (den > 0.0 ? sqrt(den) : 1.0);
            if (e > aerr) aerr = e;
        }
        /* back substitution on the rotated triangle, then x += M^-1 V y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < k; ++q) s -= H[i * m + q] * yv[q];
            yv[i] = s / H[i * m + i];
        }
        memset(z, 0, sizeof(double) * n);
        for (int i = 0; i < k; ++i)
            for (int64_t q = 0; q < n; ++q) z[q] += yv[i] * V[(int64_t)i * n + q];
        if (precond) for (int64_t q = 0; q < n; ++q) z[q] /= dg[q];
        for (int64_t q = 0; q < n; ++q) x[q] += z[q];
    }
    if (info) { info[0] = it; info[1] = restarts; info[2] = status; }
    if (dinfo) dinfo[0] = relres;
    if (arnoldi_err) *arnoldi_err = aerr;
    free(V); free(H); free(H0); free(cs); free(sn); free(g); free(yv); free(w); free(z); free(r); free(dg);
    free(samp); free(hc); free(hc2);
    if (policy_out) { policy_out[0] = faults; policy_out[1] = ortho; }
    return status;
}

int orc_gmres(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
              const double *b, double *x, int m, double tol, int64_t maxiter, int precond,
              int64_t *info, double *dinfo, double *resid_hist, double *arnoldi_err) {
    return orc_gmres_at(n, rowptr, colind, val, b, x, m, m, 0, 0.0, tol, maxiter, precond, info, dinfo,
                        resid_hist, arnoldi_err, NULL, ORC_MGS, NULL);
}

/* BiCGStab (van der Vorst 1992), right preconditioned by M = diag(A) when
 * precond == 1.  Breakdown (status 2) when rho, <rhat, v> or omega is 0.
 * Stops on the recurrence residual; the returned relative residual is the
 * true one, ||b - A x|| / ||b||. */
int orc_bicgstab(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 const double *b, double *x, double tol, int64_t maxiter, int precond, int64_t *info,
                 double *dinfo, double *resid_hist) {
    double *r = malloc(sizeof(double) * n), *rh = malloc(sizeof(double) * n);
    double *p = calloc((size_t)n, sizeof(double)), *v = calloc((size_t)n, sizeof(double));
    double *ph = malloc(sizeof(double) * n), *s = malloc(sizeof(double) * n);
    double *sh = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
    double *dg = malloc(sizeof(double) * n);
    if (precond) diag_of(n, rowptr, colind, val, dg);
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    spmv_plain(n, rowptr, colind, val, x, r);
    for (int64_t i = 0; i < n; ++i) { r[i] = b[i] - r[i]; rh[i] = r[i]; }
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    int64_t it = 0;
    int status = 1;
    double res = sqrt(dot(n, r, r)) / bn;
    if (resid_hist) resid_hist[0] = res;
    if (res <= tol) status = 0;
    while (status == 1 && it < maxiter) {
        double rho = dot(n, rh, r);
        if (rho == 0.0) { status = 2; break; }
        if (it == 0) memcpy(p, r, sizeof(double) * n);
        else {
            double beta = (rho / rho_prev) * (alpha / omega);
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        for (int64_t i = 0; i < n; ++i) ph[i] = precond ? p[i] / dg[i] : p[i];
        spmv_plain(n, rowptr, colind, val, ph, v);
        double rv = dot(n, rh, v);
        if (rv == 0.0) { status = 2; break; }
        alpha = rho / rv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        ++it;
        double sres = sqrt(dot(n, s, s)) / bn;
        if (sres <= tol) {
            for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            if (resid_hist) resid_hist[it] = sres;
            status = 0;
            break;
        }
        for (int64_t i = 0; i < n; ++i) sh[i] = precond ? s[i] / dg[i] : s[i];
        spmv_plain(n, rowptr, colind, val, sh, t);
        double tt = dot(n, t, t);
        if (tt == 0.0) { status = 2; break; }
        omega = dot(n, t, s) / tt;
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i] + omega * sh[i];
        for (int64_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        res = sqrt(dot(n, r, r)) / bn;
        if (resid_hist) resid_hist[it] = res;
        if (res <= tol) { status = 0; break; }
        if (omega == 0.0) { status = 2; break; }
        rho_prev = rho;
    }
    spmv_plain(n, rowptr, colind, val, x, t);
    for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    if (info) { info[0] = it; info[1] = 0; info[2] = status; }
    if (dinfo) dinfo[0] = sqrt(dot(n, t, t)) / bn;
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(dg);
    return status;
}
