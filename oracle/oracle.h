/*
 * CPU oracle for the auto-tuned CSR SpMV / Krylov path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this library: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Plain, serial, FP64.  Each routine follows the passage of the paper (or
 * the textbook definition) named in its comment; where the paper leaves a
 * detail open, the reading taken is stated there.
 *
 * Parity status per routine:
 *   orc_spmv_csr / orc_spmv_rows    pinned (dense matvec, integer exactness,
 *                                   stencil closed forms, eigenpairs)
 *   orc_sym_expand / orc_spmv_sym   pinned (full-storage generator, counts)
 *   orc_plan_*                      pinned (linear-scan brute force)
 *   orc_features_stats              pinned (independent numpy statistics)
 *   orc_mlp_*                       pinned (finite differences, closed forms)
 *   orc_gmres                       pinned (identity, diagonal, eigenvector,
 *                                   Arnoldi relation, direct solve)
 *   orc_bicgstab                    pinned (identity, direct solve, the 2x2
 *                                   rotation breakdown); the paper's modified
 *                                   BiCGStab variant is not described in it:
 *                                   that modification is parity unpinned.
 */
#ifndef XAB_ORACLE_H
#define XAB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y_i = sum_k val_k x_{col_k} (Dot2 compensated), s_i = sum_k |val_k x_{col_k}| */
void orc_spmv_csr(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                  const double *x, double *y, double *s);
void orc_spmv_rows(int64_t nsample, const int64_t *rows, const int32_t *rowptr,
                   const int32_t *colind, const double *val, const double *x, double *y, double *s);

/* Lower-triangle storage -> full storage A = L + L_strict^T.
 * Returns nnz_full; with null outputs only counts. */
int64_t orc_sym_expand(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                       int32_t *rowptr_f, int32_t *colind_f, double *val_f);
/* y = (L + L_strict^T) x by expansion, s over the full row */
int orc_spmv_sym(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 const double *x, double *y, double *s);

/* Plans (integer, bit-exact definitions) */
int64_t orc_nparts(int64_t nnz, int64_t T);
void orc_plan_nnz(int64_t n, const int32_t *rowptr, int64_t P, int32_t *b);
void orc_plan_bss(int64_t n, const int32_t *rowptr, int64_t T, int64_t P, int32_t *row_lo,
                  int32_t *tile_row, int32_t *carry_row);
int64_t orc_plan_sym_ntiles(int64_t n, const int32_t *rowptr, int64_t T, int64_t Rmax);
void orc_plan_sym_tiles(int64_t n, const int32_t *rowptr, int64_t T, int64_t Rmax, int32_t *b);
int64_t orc_plan_sym_touch(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t P,
                           const int32_t *b, int64_t C, int32_t *tm_ptr, int32_t *tm_tile,
                           int32_t *tile_ptr, int32_t *tile_blk, int32_t *tile_slot);

/* Column-blocked split: block k holds columns [floor(k*ncols/nb),
 * floor((k+1)*ncols/nb)).  rp[k*(n+1) + i] = entries of block k in rows < i
 * (so rp[k*(n+1) + n] = block size); ci = the column indices of block 0 in
 * row order (original order inside a row), then block 1, and so on. */
void orc_plan_xcb(int64_t n, int64_t ncols, const int32_t *rowptr, const int32_t *colind, int nb, int32_t *rp,
                  int32_t *ci);
void orc_xcb_flag_heads(int64_t n, int nb, const int32_t *rp, int32_t *ci);
int64_t orc_plan_sym_slices(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t P, const int32_t *b,
                            int64_t lanes, int32_t *ch0, int32_t *cw, int64_t *coff, int32_t *cols, int64_t *nch,
                            int64_t *widest);
int orc_sym_walk_sliced(int64_t nnz, int64_t padded, int64_t widest);
void orc_plan_sym_colflags(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t P, const int32_t *b,
                           int64_t lanes, int64_t J, int32_t *out);
int64_t orc_plan_sell(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, int C,
                      int sigma, int32_t *perm, int64_t *cptr, int32_t *clen, int32_t *rlen, int32_t *cols,
                      double *vals);
/* Block CSR with b x b blocks (section 5 leaves BCSR to future work): block
 * row R holds rows [bR, min(bR + b, n)); its blocks are the distinct c / b of
 * its entries, ascending; a block stores b*b values row-major (0 where the
 * matrix has no entry, duplicates summed in CSR order) and a mask with bit
 * (r % b) * b + c % b set for every stored position.  Returns the number of
 * blocks; brp[nbr + 1], bci, bmask and bval may be NULL (count only). */
int64_t orc_plan_bcsr(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, int b,
                      int64_t *brp, int32_t *bci, uint32_t *bmask, double *bval);

/* Selector features: integer statistics then the 12 features. */
void orc_features(int64_t n, const int32_t *rowptr, const int32_t *colind, int sym_lower,
                  int64_t *stats, double *feat);

/* MLP 12-H-H-K (ReLU) in FP64.  Flat parameter layout:
 * W1[H*F] b1[H] W2[H*H] b2[H] W3[K*H] b3[K], row-major (out, in). */
int64_t orc_mlp_nparams(int F, int H, int K);
void orc_mlp_forward(int F, int H, int K, const double *p, int64_t B, const double *feat, double *out);
double orc_mlp_loss_grad(int F, int H, int K, const double *p, int64_t B, const double *feat,
                         const double *y, const uint8_t *mask, double *grad);
void orc_adam_step(int64_t np, double *p, const double *g, double *m, double *v, int64_t t, double lr,
                   double b1, double b2, double eps);
void orc_mlp_train(int F, int H, int K, double *p, int64_t M, const double *feat, const double *y,
                   const uint8_t *mask, const int32_t *order, int epochs, int batch, double lr,
                   double *loss_per_epoch);

/* Krylov solvers.  precond: 0 none, 1 right Jacobi.
 * info[0] iterations, info[1] restarts, info[2] status (0 ok, 1 not
 * converged, 2 breakdown); dinfo[0] final true relative residual.
 * resid_hist (optional, length maxiter+1) receives the recurrence residual
 * estimate after every Arnoldi step / iteration, relative to ||b||. */
int orc_gmres(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
              const double *b, double *x, int m, double tol, int64_t maxiter, int precond,
              int64_t *info, double *dinfo, double *resid_hist, double *arnoldi_err);
double orc_mm_ratio(const double *r, int64_t s, int64_t t);
/* ortho: 0 DGKS, 1 CGS, 2 MGS, 3 BCGS (block 4), 4 the accuracy policy;
 * policy_out (may be NULL) receives [faults, final ortho]. */
int orc_gmres_at(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 const double *b, double *x, int m0, int m_max, int step, double ratio, double tol,
                 int64_t maxiter, int precond, int64_t *info, double *dinfo, double *resid_hist,
                 double *arnoldi_err, int32_t *m_hist, int ortho, int32_t *policy_out);
int orc_bicgstab(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 const double *b, double *x, double tol, int64_t maxiter, int precond, int64_t *info,
                 double *dinfo, double *resid_hist);

#ifdef __cplusplus
}
#endif
#endif
