/*
 * Seeded synthetic input generators (test and benchmark fixtures).
 *
 * These build CSR matrices and vectors shaped like the workloads of the
 * paper's evaluation (section 4.2 and 4.4): stencil/FEM-like symmetric
 * matrices, unbalanced unsymmetric ones, a trans4-shaped stress matrix, a
 * batch of uneven systems and the learned-selector training families.  They
 * hold none of the method's arithmetic (no product, no reduction of A*x):
 * they only write rowptr / colind / val / x arrays.  Both the CPU oracle and
 * the GPU path are fed from here.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood 2014), counter based.
 * Every row (or element) owns a substream keyed by (seed, id), so the output
 * does not depend on the number of OpenMP threads.
 *   U(0,1)  = top 53 bits * 2^-53
 *   N(0,1)  = Box-Muller, cosine branch only, u1 taken as 1 - U so that
 *             log() never sees 0.
 *
 * Every fill routine is two-phase: a *_lengths() call writes row lengths,
 * the caller turns them into rowptr (prefix sum, checked against 2^31), and
 * a *_fill() call writes colind (sorted ascending per row) and val.
 *
 * Diagonal rule for generated dominant matrices: a_ii = 1.1 * sum_{j != i}
 * |a_ij| over the FULL row, or 1.0 when that sum is 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define XG_GOLDEN 0x9E3779B97F4A7C15ULL

typedef struct { uint64_t s; } xg_rng;

static inline uint64_t xg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline void xg_seed(xg_rng *r, uint64_t seed, uint64_t id) {
    r->s = xg_mix(seed ^ 0x5851F42D4C957F2DULL) ^ xg_mix(id + 0x14057B7EF767814FULL);
}

static inline uint64_t xg_next(xg_rng *r) {
    r->s += XG_GOLDEN;
    return xg_mix(r->s);
}

static inline double xg_u01(xg_rng *r) { return (double)(xg_next(r) >> 11) * 0x1.0p-53; }

static inline double xg_normal(xg_rng *r) {
    double u1 = 1.0 - xg_u01(r);
    double u2 = xg_u01(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

/* uniform integer in [lo, hi] inclusive (hi - lo < 2^53) */
static inline int64_t xg_uint(xg_rng *r, int64_t lo, int64_t hi) {
    double u = xg_u01(r);
    int64_t v = lo + (int64_t)floor(u * (double)(hi - lo + 1));
    return v > hi ? hi : v;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Exported: the SplitMix64 streams themselves, so tests can check them. */
uint64_t xg_stream_u64(uint64_t seed, uint64_t id, int64_t k) {
    xg_rng r;
    xg_seed(&r, seed, id);
    uint64_t v = 0;
    for (int64_t i = 0; i <= k; ++i) v = xg_next(&r);
    return v;
}

/* out[i] = lo + (hi - lo) * U, one substream per element */
void xg_uniform_vec(int64_t n, uint64_t seed, double lo, double hi, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        xg_rng r;
        xg_seed(&r, seed, (uint64_t)i);
        out[i] = lo + (hi - lo) * xg_u01(&r);
    }
}

/* integer-valued vector in [lo, hi] (for exact-arithmetic pins) */
void xg_int_vec(int64_t n, uint64_t seed, int32_t lo, int32_t hi, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        xg_rng r;
        xg_seed(&r, seed, (uint64_t)i);
        out[i] = (double)xg_uint(&r, lo, hi);
    }
}

/* ---------------------------------------------------------------------
 * Stencils on a g^dim grid, Dirichlet truncation, lexicographic order
 * (x fastest).  npts: dim 2 -> 5 or 9, dim 3 -> 7 or 27.
 * lower != 0 keeps j <= i only (the diagonal included).
 * Values: off-diagonals offval; diagonal diagval, or, if diag_dominant,
 * 1.1 * (number of off-diagonals in the full row) * |offval|.
 * ------------------------------------------------------------------- */
static int stencil_offsets(int dim, int npts, int off[27][3]) {
    int k = 0;
    for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int nz = (dx != 0) + (dy != 0) + (dz != 0);
                int keep;
                if (npts == 5 || npts == 7) keep = nz <= 1;
                else keep = 1; /* 9 or 27 */
                if (!keep) continue;
                off[k][0] = dx; off[k][1] = dy; off[k][2] = dz;
                ++k;
            }
    return k; /* already in ascending column order for lexicographic index */
}

static int stencil_valid(int dim, int npts) {
    return (dim == 2 && (npts == 5 || npts == 9)) || (dim == 3 && (npts == 7 || npts == 27));
}

int xg_stencil_lengths(int dim, int npts, int32_t g, int lower, int32_t *len) {
    if (!stencil_valid(dim, npts) || g < 1) return -1;
    int off[27][3];
    int m = stencil_offsets(dim, npts, off);
    int64_t n = (int64_t)g * g * (dim == 3 ? g : 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t x = i % g, y = (i / g) % g, z = (dim == 3) ? i / ((int64_t)g * g) : 0;
        int c = 0;
        for (int k = 0; k < m; ++k) {
            int64_t xx = x + off[k][0], yy = y + off[k][1], zz = z + off[k][2];
            if (xx < 0 || xx >= g || yy < 0 || yy >= g || zz < 0 || zz >= (dim == 3 ? g : 1)) continue;
            int64_t j = xx + (int64_t)g * (yy + (int64_t)g * zz);
            if (lower && j > i) continue;
            ++c;
        }
        len[i] = c;
    }
    return 0;
}

int xg_stencil_fill(int dim, int npts, int32_t g, int lower, double diagval, double offval,
                    int diag_dominant, const int32_t *rowptr, int32_t *colind, double *val) {
    if (!stencil_valid(dim, npts) || g < 1) return -1;
    int off[27][3];
    int m = stencil_offsets(dim, npts, off);
    int64_t n = (int64_t)g * g * (dim == 3 ? g : 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t x = i % g, y = (i / g) % g, z = (dim == 3) ? i / ((int64_t)g * g) : 0;
        int64_t p = rowptr[i];
        int nfull_off = 0;
        for (int k = 0; k < m; ++k) {
            int64_t xx = x + off[k][0], yy = y + off[k][1], zz = z + off[k][2];
            if (xx < 0 || xx >= g || yy < 0 || yy >= g || zz < 0 || zz >= (dim == 3 ? g : 1)) continue;
            int64_t j = xx + (int64_t)g * (yy + (int64_t)g * zz);
            if (j != i) ++nfull_off;
            if (lower && j > i) continue;
            colind[p] = (int32_t)j;
            val[p] = (j == i) ? 0.0 : offval;
            ++p;
        }
        double d = diag_dominant ? (nfull_off ? 1.1 * nfull_off * fabs(offval) : 1.0) : diagval;
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            if (colind[q] == i) val[q] = d;
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Row-length laws.
 * ------------------------------------------------------------------- */

/* len_i = clip(round(exp(N(mu, sigma))), lmin, lmax); draws are the first
 * two uniforms of row i's substream. */
void xg_lognormal_lengths(int64_t n, uint64_t seed, double mu, double sigma, int32_t lmin,
                          int32_t lmax, int32_t *len) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        xg_rng r;
        xg_seed(&r, seed, (uint64_t)i);
        double v = round(exp(mu + sigma * xg_normal(&r)));
        if (v < lmin) v = lmin;
        if (v > lmax) v = lmax;
        len[i] = (int32_t)v;
    }
}

/* len_i ~ U{lmin..lmax} (first uniform of row i's substream) */
void xg_uniform_lengths(int64_t n, uint64_t seed, int32_t lmin, int32_t lmax, int32_t *len) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        xg_rng r;
        xg_seed(&r, seed, (uint64_t)i);
        len[i] = (int32_t)xg_uint(&r, lmin, lmax);
    }
}

/* trans4-shaped law: row `long_row` has `long_len`; every other row has a
 * length in [1, 7], the total being exactly `total`.  Start from U{1..7},
 * then walk a dedicated substream adding/removing one entry at a time. */
int xg_trans4_lengths(int64_t n, uint64_t seed, int64_t long_row, int32_t long_len, int64_t total,
                      int32_t *len) {
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) {
        xg_rng r;
        xg_seed(&r, seed, (uint64_t)i);
        len[i] = (i == long_row) ? long_len : (int32_t)xg_uint(&r, 1, 7);
        s += len[i];
    }
    int64_t lo = long_len + (n - 1), hi = long_len + 7 * (n - 1);
    if (total < lo || total > hi) return -1;
    xg_rng r;
    xg_seed(&r, seed, 0xFFFFFFFFFFFFULL);
    while (s != total) {
        int64_t i = xg_uint(&r, 0, n - 1);
        if (i == long_row) continue;
        if (s < total && len[i] < 7) { ++len[i]; ++s; }
        else if (s > total && len[i] > 1) { --len[i]; --s; }
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Random rows: row i holds its diagonal plus len_i - 1 distinct columns
 * drawn uniformly from [0, ncols) \ {i}, sorted.  Off-diagonal values
 * N(0,1) in sorted-column order; diagonal by the dominance rule.  The row
 * substream is the same one the length law used (seed, i), continued after
 * skip_draws uniforms so lengths and contents never share draws.
 * If with_diag == 0 (non-square use) all len_i columns are random.
 * ------------------------------------------------------------------- */
static void sample_distinct(xg_rng *r, int64_t m, int64_t k, int32_t *out, unsigned char *mark) {
    /* k distinct values from [0, m), unsorted on return */
    if (k == 0) return;
    if (k * 4 > m && mark) {
        /* Floyd's algorithm with a bitmap */
        memset(mark, 0, (size_t)m);
        int64_t c = 0;
        for (int64_t j = m - k; j < m; ++j) {
            int64_t t = xg_uint(r, 0, j);
            if (mark[t]) t = j;
            mark[t] = 1;
            out[c++] = (int32_t)t;
        }
        return;
    }
    int64_t have = 0;
    while (have < k) {
        for (int64_t c = have; c < k; ++c) out[c] = (int32_t)xg_uint(r, 0, m - 1);
        qsort(out, (size_t)k, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t c = 0; c < k; ++c)
            if (c == 0 || out[c] != out[u - 1]) out[u++] = out[c];
        have = u;
    }
}

int xg_random_rows_fill(int64_t n, int64_t ncols, uint64_t seed, int skip_draws, int with_diag,
                        const int32_t *rowptr, int32_t *colind, double *val) {
    int32_t maxlen = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t l = rowptr[i + 1] - rowptr[i];
        if (l > maxlen) maxlen = l;
    }
    int bad = 0;
#pragma omp parallel
    {
        unsigned char *mark = (unsigned char *)malloc((size_t)(ncols > 0 ? ncols : 1));
        int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxlen + 1));
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            xg_rng r;
            xg_seed(&r, seed, (uint64_t)i);
            for (int d = 0; d < skip_draws; ++d) xg_next(&r);
            int64_t p0 = rowptr[i], len = rowptr[i + 1] - rowptr[i];
            if (len == 0) continue;
            int64_t k = with_diag ? len - 1 : len;
            int64_t m = with_diag ? ncols - 1 : ncols;
            if (k > m) { bad = 1; continue; }
            sample_distinct(&r, m, k, tmp, mark);
            if (with_diag)
                for (int64_t c = 0; c < k; ++c)
                    if (tmp[c] >= i) tmp[c] += 1; /* skip the diagonal */
            if (with_diag) tmp[k] = (int32_t)i;
            qsort(tmp, (size_t)len, sizeof(int32_t), cmp_i32);
            double asum = 0.0;
            for (int64_t c = 0; c < len; ++c) {
                colind[p0 + c] = tmp[c];
                if (with_diag && tmp[c] == i) { val[p0 + c] = 0.0; continue; }
                double v = xg_normal(&r);
                val[p0 + c] = v;
                asum += fabs(v);
            }
            if (with_diag)
                for (int64_t c = 0; c < len; ++c)
                    if (colind[p0 + c] == i) val[p0 + c] = asum > 0.0 ? 1.1 * asum : 1.0;
        }
        free(mark);
        free(tmp);
    }
    return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------
 * Banded: dense band |i - j| <= h.  lower != 0 keeps j <= i (symmetric
 * lower storage; the dominance rule then uses the full symmetric row).
 * Value of entry (i, j), j < i, drawn from row i's substream in column
 * order; for general storage the upper entries (j > i) come after.
 * ------------------------------------------------------------------- */
void xg_banded_lengths(int64_t n, int32_t h, int lower, int32_t *len) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = i - h < 0 ? 0 : i - h;
        int64_t hi = lower ? i : (i + h > n - 1 ? n - 1 : i + h);
        len[i] = (int32_t)(hi - lo + 1);
    }
}

void xg_banded_fill(int64_t n, int32_t h, int lower, uint64_t seed, const int32_t *rowptr,
                    int32_t *colind, double *val) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        xg_rng r;
        xg_seed(&r, seed, (uint64_t)i);
        int64_t lo = i - h < 0 ? 0 : i - h;
        int64_t p = rowptr[i];
        double asum = 0.0;
        for (int64_t j = lo; j < i; ++j) { /* strictly lower part first */
            colind[p] = (int32_t)j;
            val[p] = xg_normal(&r);
            asum += fabs(val[p]);
            ++p;
        }
        int64_t pd = p;
        colind[p] = (int32_t)i; val[p] = 0.0; ++p;
        if (!lower) {
            int64_t hi = i + h > n - 1 ? n - 1 : i + h;
            for (int64_t j = i + 1; j <= hi; ++j) {
                colind[p] = (int32_t)j;
                val[p] = xg_normal(&r);
                asum += fabs(val[p]);
                ++p;
            }
            val[pd] = asum > 0.0 ? 1.1 * asum : 1.0;
        } else {
            val[pd] = asum; /* completed below with the column part */
        }
    }
    if (lower) {
        /* add the transposed part of each symmetric row: column sums of |L_strict| */
        double *cs = (double *)calloc((size_t)n, sizeof(double));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rowptr[i]; p < rowptr[i + 1] - 1; ++p) cs[colind[p]] += fabs(val[p]);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t pd = rowptr[i + 1] - 1; /* diagonal is last in a lower row */
            double s = val[pd] + cs[i];
            val[pd] = s > 0.0 ? 1.1 * s : 1.0;
        }
        free(cs);
    }
}

/* ---------------------------------------------------------------------
 * Block-diagonal with dense blocks, sizes U{bmin..bmax} drawn in sequence
 * from substream (seed, 2^48 - 1); the last block is cut at n.
 * blk_start must have room for n + 1 entries; returns the block count.
 * ------------------------------------------------------------------- */
int64_t xg_blockdiag_blocks(int64_t n, uint64_t seed, int32_t bmin, int32_t bmax, int64_t *blk_start) {
    xg_rng r;
    xg_seed(&r, seed, 0xFFFFFFFFFFFFULL);
    int64_t nb = 0, s = 0;
    while (s < n) {
        blk_start[nb++] = s;
        s += xg_uint(&r, bmin, bmax);
    }
    blk_start[nb] = n;
    return nb;
}

void xg_blockdiag_lengths(int64_t nb, const int64_t *blk_start, int32_t *len) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t i = blk_start[b]; i < blk_start[b + 1]; ++i)
            len[i] = (int32_t)(blk_start[b + 1] - blk_start[b]);
}

void xg_blockdiag_fill(int64_t nb, const int64_t *blk_start, uint64_t seed, const int32_t *rowptr,
                       int32_t *colind, double *val) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t i = blk_start[b]; i < blk_start[b + 1]; ++i) {
            xg_rng r;
            xg_seed(&r, seed, (uint64_t)i);
            int64_t p = rowptr[i], pd = -1;
            double asum = 0.0;
            for (int64_t j = blk_start[b]; j < blk_start[b + 1]; ++j, ++p) {
                colind[p] = (int32_t)j;
                if (j == i) { pd = p; val[p] = 0.0; continue; }
                val[p] = xg_normal(&r);
                asum += fabs(val[p]);
            }
            val[pd] = asum > 0.0 ? 1.1 * asum : 1.0;
        }
}

/* ---------------------------------------------------------------------
 * Batch of uneven systems.  System k is keyed by sid = seed * 2^32 + k;
 * its parameters come from substream (sid, 2^48 - 1):
 *   n_k = round(exp(U(ln nmin, ln nmax)))
 *   banded (k even): half-bandwidth h ~ U{1..hmax}
 *   random (k odd):  row lengths U{lmin..lmax}, diagonal included
 * ------------------------------------------------------------------- */
void xg_batch_params(int32_t nsys, uint64_t seed, double nmin, double nmax, int32_t hmax,
                     int32_t *n_out, int32_t *kind_out, int32_t *h_out) {
    for (int32_t k = 0; k < nsys; ++k) {
        uint64_t sid = seed * 4294967296ULL + (uint64_t)k;
        xg_rng r;
        xg_seed(&r, sid, 0xFFFFFFFFFFFFULL);
        double u = xg_u01(&r);
        n_out[k] = (int32_t)round(exp(log(nmin) + u * (log(nmax) - log(nmin))));
        kind_out[k] = (k % 2 == 0) ? 0 : 1;
        int32_t h = (int32_t)xg_uint(&r, 1, hmax);
        h_out[k] = kind_out[k] == 0 ? h : 0;
    }
}

uint64_t xg_batch_sid(uint64_t seed, int32_t k) { return seed * 4294967296ULL + (uint64_t)k; }
